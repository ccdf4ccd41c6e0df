/*
 * dsvof -- one GPU (gfx950) time step of a VOF droplet-evaporation method:
 * liquid-fraction transport with an interface evaporation source, implicit
 * energy and vapour-species diffusion, and a variable-density pressure
 * projection with gravity and a centripetal body force.
 *
 * Method: arXiv 2005.02867 (DropletSMOKE++), Sections 2-3.  The step follows
 * the segregated order of Section 3.1 (evaporation flux, liquid source,
 * interface advection, properties, momentum/energy/species, pressure and
 * velocity correction), discretised on a uniform Cartesian grid.
 *
 * Grid and layout (all arrays are device pointers, IEEE binary64, dense):
 *   cells (i, j, k), 0 <= i < nx ..., spacing h, centre ((i+.5)h, (j+.5)h, (k+.5)h);
 *   cell array index  (i*ny + j)*nz + k          (z fastest)
 *   u: (nx+1)*ny*nz   index (i*ny + j)*nz + k    (face i at x = i h)
 *   v: nx*(ny+1)*nz   index (i*(ny+1) + j)*nz + k
 *   w: nx*ny*(nz+1)   index (i*ny + j)*(nz+1) + k
 * Boundaries (boundary-condition table of Section 3.2 mapped onto the box):
 *   z- inlet, z+ outlet, x-/x+/y-/y+ outer wall; bc_mode selects natural or
 *   forced convection, or an all-open far field.
 *
 * Memory ownership: the library never allocates device memory.  All device
 * state lives in one caller-owned workspace of ds_workspace_bytes() bytes
 * that must stay allocated and untouched while the handle uses it.  Field
 * arrays passed to set/get are copied (device to device) on the given
 * stream.  The library owns only the host handle (and a small pinned host
 * buffer for scalars).
 *
 * Streams: every call enqueues work on `stream` (a hipStream_t; NULL means
 * the null stream).  Calls that return host scalars synchronise that stream.
 * A step may also run part of its work on a stream of the handle's own
 * (DSVOF_OVERLAP below); it forks from `stream` with an event and `stream`
 * waits for it with another before the step's next stage, so every call's
 * work is ordered on `stream` as a whole.
 *
 * Errors: every call returns a ds_status; ds_last_error() gives a message.
 * No call throws.  A handle is not thread-safe.
 */
#ifndef DSVOF_H
#define DSVOF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ds_grid ds_grid;

typedef enum ds_status {
  DS_OK = 0,
  DS_ERR_ARG = -1,            /* invalid argument (nothing was changed)          */
  DS_ERR_HIP = -2,            /* a HIP runtime call failed                        */
  DS_ERR_NOT_CONVERGED = -3,  /* a linear solve hit maxit; the state advanced with
                                 the last iterate; see ds_get_diagnostics()        */
  DS_ERR_NONFINITE = -4,      /* a non-finite value appeared; state unspecified,
                                 restore it with ds_set_fields()                   */
  DS_ERR_STATE = -5           /* call out of order (e.g. step before set_fields)  */
} ds_status;

enum { DS_EQ_IDEAL = 0, DS_EQ_PENG_ROBINSON = 1 };
enum { DS_BC_NATURAL = 0, DS_BC_FORCED = 1, DS_BC_FARFIELD = 2 };
enum { DS_PREC_FP64 = 0, DS_PREC_MIXED = 1 };
/* Species forms (Section 2.5).  CONSERVATIVE: vapour lives in the gas
 * fraction, c = rho_G theta omega gains mdot and is updated in flux form, the
 * flux at adj is rho_G D (omega_sat(T_int) - omega_adj)/d.  LITERAL: the
 * saturation value omega_sat(T) is assigned to every liquid cell
 * (alpha > eps_gas) at the start of a step, the diffusive flux at adj is
 * -rho_G D grad(omega).n with a central gradient (zero-gradient ghosts), and
 * the species equation (eq. 9) has no mdot source; not mass conserving. */
enum { DS_SPECIES_CONSERVATIVE = 0, DS_SPECIES_LITERAL = 1 };
/* Gas density (Section 2.5, eq. 24; Section 2.2, eq. 7).  AMBIENT: one value,
 * eq. 24 for the ambient gas at (T_amb, p), in every cell.  VARIABLE: eq. 24
 * per cell for the local fuel/N2 mixture (mole fraction from omega; Z = 1 or
 * the Peng-Robinson root of the mixture with the equilibrium's mixing rules).
 * The state's c and T then fix omega and rho_G (rho_G omega = c/theta); a
 * step uses the start-of-step rho_G for the interface flux and the vapour
 * flux (face value of rho_G omega), the advected state's rho_G' for the
 * properties, the species system (cell coefficient rho_G' theta, Dirichlet
 * faces at the ambient gas), the predictor and the pressure, and adds eq. 7's
 * -(1 - alpha')(1/rho_G) D rho_G/Dt = -(1 - alpha') ln(rho_G^{n+1}/rho_G')/dt
 * to the pressure source.  Not with the literal species form or the
 * differentiation form. */
enum { DS_GAS_AMBIENT = 0, DS_GAS_VARIABLE = 1 };
/* Liquid advection (Section 2.1, eq. 3).  FLUX_LIMITED: TVD van Leer face
 * values.  GEOMETRIC: the paper's choice of a geometric scheme (isoAdvector),
 * with a plane per surface cell (1e-8 < alpha1 < 1 - 1e-8): normal
 * -grad(alpha1)/|grad(alpha1)| by central differences (ghosts repeat the
 * boundary cell), offset leaving alpha1 h^3 of liquid; the liquid through a
 * face in the step is the face velocity times the time integral of the area
 * the donor cell's plane submerges while it moves with the donor's centre
 * velocity along the normal (exact piecewise integration); other donors give
 * U_f alpha1 dt; no bounding step (the update stays conservative).  The
 * vapour and temperature fluxes keep the flux-limited face values.  Not with
 * the differentiation form. */
enum { DS_ADV_FLUX_LIMITED = 0, DS_ADV_GEOMETRIC = 1 };

/* Physical and numerical parameters, SI units.  Property values are constant
 * (the mixing rule of Section 2.7, eq. 31, blends liquid and gas values). */
typedef struct ds_params {
  double h;            /* grid spacing [m] */
  double dt;           /* time step [s] */
  double p;            /* thermodynamic pressure [Pa] */
  double T_amb;        /* ambient gas temperature [K] (boundary value) */
  double rho_L, cp_L, k_L;   /* liquid density, heat capacity, conductivity */
  double cp_G, k_G;          /* gas heat capacity, conductivity */
  double D_v;          /* vapour diffusivity in the gas [m^2/s] */
  double dh_ev;        /* latent heat [J/kg] (energy sink and Clausius-Clapeyron) */
  double M_v, M_G;     /* molar masses of fuel and ambient gas [kg/mol] */
  double g[3];         /* gravity [m/s^2] */
  double xi0;          /* centripetal potential intensity [m^2/s^2] (eq. 29) */
  double Df;           /* fiber length scale in eq. 29 [m] */
  double r_fib;        /* radius below which the potential is held constant [m] */
  double w_in;         /* forced inflow velocity at z- [m/s] */
  double x0[3];        /* droplet / fiber centre; origin of g.r [m] */
  double Tc, Pc, acentric;         /* fuel critical data (Peng-Robinson) */
  double Tc_G, Pc_G, acentric_G;   /* ambient gas critical data */
  double kij;          /* binary interaction coefficient */
  double T_ref, p_ref; /* Clausius-Clapeyron reference point */
  double eps_int;      /* interface-cell threshold on alpha */
  double eps_gas;      /* a cell with alpha <= eps_gas counts as gas for the adj march */
  double theta_min;    /* lower bound of the gas fraction in the species system */
  double tol;          /* relative residual tolerance of the linear solves */
  double tol_phi;      /* tolerance of the liquid-transport potential solve */
  int s_max;           /* longest interface-normal march, in cell lengths */
  int maxit;           /* iteration cap of each linear solve */
  int eq_model;        /* DS_EQ_* */
  int bc_mode;         /* DS_BC_* */
  int precision;       /* DS_PREC_*: FP64 solves, or FP32 sweeps + FP64 refinement */
  int solve_energy;    /* 0: temperature frozen (isothermal runs) */
  int evaporation;     /* 0: no evaporation source */
  int pressure_precond; /* 0: Jacobi-PCG, 1: geometric-multigrid PCG */
  int liquid_transport; /* 1: alpha moves with the divergence-free part of u (default); 0: with u */
  int species_form;    /* DS_SPECIES_* */
  int viscous;         /* 1: implicit viscous momentum, div mu (grad v + grad v^T) of eqs. 5 and 30 (0: mu = 0) */
  double mu_L, mu_G;   /* liquid and gas dynamic viscosity [Pa s], mixed by eq. 31 (used with viscous = 1) */
  int gas_density;     /* DS_GAS_*: the gas density of eq. 24 */
  int advection;       /* DS_ADV_*: the liquid advection of eq. 3 */
} ds_params;

/* Scalars of the most recent step (or evaporation/pressure call). */
typedef struct ds_diagnostics {
  double K;              /* redistribution constant of eq. 20 */
  double mdot_total;     /* h^3 sum(mdot) [kg/s] */
  double volume;         /* h^3 sum(alpha) [m^3] */
  double fuel_mass;      /* h^3 sum(rho_L alpha + c) after the step [kg] */
  double fuel_mass_before;
  double B_L, B_v;       /* liquid / vapour mass that left the box during the step [kg] */
  double alpha_min, alpha_max;
  double res_T, res_omega, res_p;   /* final relative residuals */
  double rho_G;          /* gas density of the ambient gas (eq. 24); with DS_GAS_VARIABLE the
                            per-cell field is DS_FIELD_RHO_G */
  int iters_T, iters_omega, iters_p;
  int n_interface;       /* interface cells with a nonzero gradient */
  int converged;         /* 1 if every solve met tol */
  int refinements_p;     /* outer FP64 refinement rounds of the pressure solve */
  int iters_phi;         /* iterations of the liquid-transport potential solve */
  double res_phi;
  int rounds_T, rounds_omega;   /* FP32 rounds of the energy and species solves (precision form; 0 in FP64) */
  int iters_visc;        /* iterations of the implicit viscous solve (viscous = 1) */
  double res_visc;
} ds_diagnostics;

/* Validate parameters and create a host handle for an nx*ny*nz grid
 * (each >= 2).  The problem statement the handle holds is the paper's: the
 * domain and boundary conditions (Section 3.2, mapped onto the box as above),
 * the constant properties and their mixing rule (Section 2.7, eq. 31), the
 * operating conditions T, p and the equilibrium model (Section 2.5, eqs.
 * 22-25), the centripetal potential's xi0 (Section 2.6, eq. 29) and the time
 * step of the segregated algorithm (Section 3.1).  The gas density is fixed
 * here from eq. 24 for the ambient gas at (T_amb, p).  Host only.  Returns
 * DS_ERR_ARG for invalid input.
 *
 * Tuning variables read from the environment here (unset: the defaults in
 * brackets, which every measurement uses).  They change launch shapes and
 * solver schedules, never the discretisation; results stay within the
 * solver tolerance.
 *   DSVOF_MG_NU [4], DSVOF_MG_NU_FINE [4]: V-cycle pre/post Jacobi sweeps
 *     (coarse levels, finest level); DSVOF_MG_COARSE [16]: sweeps on the
 *     coarsest level; DSVOF_MG_MINDIM [8]: coarsen while every side is at
 *     least this; DSVOF_MG_OMEGA [0.9]: Jacobi damping; DSVOF_MG_TAIL [1]:
 *     run the levels that fit in LDS in one workgroup; DSVOF_MG_RB [1]:
 *     coloured (x-z red-black) sweeps on the levels that take them, with
 *     DSVOF_MG_RB_NU [3] pre/post sweeps, weight DSVOF_MG_RB_W [1.0], on
 *     levels whose marching chunks have at least DSVOF_MG_RB_MINPLANES [8]
 *     x-planes.
 *   DSVOF_INNER_MIN [1e-3], DSVOF_INNER_MIN_JAC [1e-6]: smallest relative
 *     reduction an FP32 round of the precision form asks (pressure-type,
 *     energy/species); DSVOF_MG32 [1]: multigrid systems of the precision
 *     form as FP64 CG with the FP32 V-cycle (0: FP32 rounds).
 *   DSVOF_NEUMANN [1]: energy and species CG preconditioned by the first-
 *     order Neumann polynomial of the Jacobi splitting (0: Jacobi).
 *   DSVOF_CONST_Q [1]: the liquid-transport potential's fine-level
 *     coloured sweep and CG operator take its constant face coefficient
 *     from a register instead of loading it (same arithmetic).
 *   DSVOF_ROUND_TEST [1]: each FP32 round of the energy and species solves
 *     enqueues its expected inner iterations and takes one host convergence
 *     test, and the solve's start takes none (0: the start and the inner
 *     solve are tested as well).
 *   DSVOF_PHI_DIRECT [1]: the liquid-transport potential by the direct solve
 *     (fast diagonalisation: DCT-II/DST-II bases along x and y, the z line
 *     solved in the same way, FFTs in LDS) wherever the grid allows it (each
 *     lateral axis with equal box faces, extents 4^a 2^b 3^c up to 1024, 2 nz
 *     for a no-flux z- face); its true FP64 residual is checked, and the
 *     multigrid CG takes over from its result should it miss tol_phi (0: the
 *     multigrid CG always).
 *   DSVOF_EXTRAP [1]: ds_step starts each species solve from omega' plus
 *     the previous step's solve correction (omega~ - omega'), kept in the
 *     workspace; ds_set_fields clears it, and ds_forward_record and
 *     ds_adjoint run without it (0: from omega' alone).
 *   DSVOF_OVERLAP [1]: with the multigrid pressure (ambient gas, inviscid
 *     step, either precision form), ds_step runs the momentum predictor and
 *     the pressure solve on a second stream of the handle's own (non-blocking,
 *     default priority), on arrays of their own in the workspace (five FP64
 *     arrays of the grid, and five FP32 or two FP64 more), concurrently with
 *     the energy and species solves on the caller's stream (recording and
 *     the adjoint's replays included); the projection waits for both.
 *     Results are the same bit for bit (0: one stream; the workspace is then
 *     smaller).
 *   DSVOF_GRAPHS [1]: the precision form's multigrid CG replays pairs of
 *     iterations as HIP graphs, captured on a stream of the handle's own and
 *     launched on the caller's (0: one launch at a time; same results bit
 *     for bit).
 *   DSVOF_VEC_BLOCKS [1024], DSVOF_VEC_YTILE [0]: grid cap and y-slab of the
 *     z-vectorised pointwise kernels; DSVOF_MARCH_THREADS [262144],
 *     DSVOF_MARCH_MIN_PLANES [1]: threads and shortest x-chunk of the
 *     marching stencil kernels; DSVOF_MARCH_NT0 ["512,256,384"],
 *     DSVOF_MARCH_NT1 ["256,512,384"]: block sizes the marching kernels try
 *     in order (0: CG operator and FP64 residual, 1: V-cycle).
 * Every variable is read once, here, into the handle: two handles of one
 * process keep their own settings (launch shapes included), whatever the
 * environment holds when the other is created. */
int ds_create_grid(int nx, int ny, int nz, const ds_params* prm, ds_grid** out);

/* Release the host handle.  The workspace is the caller's. */
int ds_destroy_grid(ds_grid* g);

/* Bytes of device workspace the handle needs (256-byte aligned base). */
size_t ds_workspace_bytes(const ds_grid* g);

/* Bind the workspace and load the state (Section 3.3: the caller builds the
 * initial fields).  alpha, T, omega, p: cell arrays; u, v, w: face arrays.
 * omega is the vapour mass fraction in the gas.  All pointers device,
 * read-only here. */
int ds_set_fields(ds_grid* g, const double* alpha, const double* T, const double* omega,
                  const double* u, const double* v, const double* w, const double* p,
                  void* workspace, size_t workspace_bytes, void* stream);

/* Copy the state out (device pointers; any may be NULL to skip): the fields
 * the paper reads back from a run (Section 4: droplet volume from alpha,
 * surface and mean droplet temperature from T, the vapour field omega and the
 * flow u, v, w, p_rgh), in the layout above. */
int ds_get_fields(ds_grid* g, double* alpha, double* T, double* omega, double* u,
                  double* v, double* w, double* p, void* stream);

/* Advance nsteps time steps (Section 3.1).  Synchronises the stream once per
 * linear solve batch to test convergence.  Diagnostics refer to the last step. */
int ds_step(ds_grid* g, int nsteps, void* stream);

/* On the current state, without advancing alpha, T or omega: evaporation
 * source (Section 2.4), momentum predictor with gravity and f_m (eq. 30),
 * pressure solve (eq. 7) and velocity correction; p and u, v, w are updated.
 * In the literal species form the liquid cells' omega and c are first set to
 * their saturation values (as in ds_evaporation_rate). */
int ds_solve_pressure(ds_grid* g, void* stream, int* iters, double* rel_res);

/* Solver check on the current state: solve one implicit system of the step,
 * A x = rhs, with the operator the step would assemble from the current
 * state (its alpha in the role of the advected alpha', its face velocities
 * for the inletOutlet switches of the open faces) and the step's solver for
 * that system (preconditioner, precision form and tolerance of the handle):
 *   DS_SYS_PRESSURE  eq. 7 with the velocity correction of eq. 30: face
 *                    coefficient dt/h^2 (1/rho)_f, p_rgh = 0 half a cell
 *                    outside open faces, no flux through walls and inlets;
 *   DS_SYS_ENERGY    eq. 8 in implicit Euler: rho cp/dt on the diagonal,
 *                    k_f/h^2 per face, ambient Dirichlet faces 2 k_G/h^2;
 *   DS_SYS_SPECIES   eq. 9 for the vapour in the gas fraction: rho_G theta/dt,
 *                    rho_G D theta_f/h^2 per face, Dirichlet faces 2 rho_G D/h^2;
 *   DS_SYS_POTENTIAL the liquid-transport potential (interface advection,
 *                    eq. 3, with the divergence-free part of u): the pressure
 *                    operator with 1/rho = 1/dt; solved to tol_phi, by the
 *                    direct solve where the grid allows it (iters 0).
 * rhs: device cell array (n doubles, read only).  x: device cell array, the
 * initial guess on entry and the solution on exit.  The solver stops on its
 * recursively updated residual, as in the step; rel_res is then the true FP64
 * relative residual ||rhs - A x||/||rhs|| of the returned x, and the call
 * returns DS_ERR_NOT_CONVERGED when it exceeds the tolerance.
 * The state (alpha, c, omega, T, p, u, v, w) is not changed; operator and
 * solver scratch of the workspace are overwritten.  Returns
 * DS_ERR_NOT_CONVERGED (x holds the last iterate) when maxit is reached or
 * the true residual misses the tolerance,
 * DS_ERR_ARG for an unknown system or null pointer, DS_ERR_STATE before
 * ds_set_fields.  Synchronises the stream. */
enum { DS_SYS_PRESSURE = 0, DS_SYS_ENERGY = 1, DS_SYS_SPECIES = 2, DS_SYS_POTENTIAL = 3 };
int ds_solve_system(ds_grid* g, int which, const double* rhs, double* x, void* stream, int* iters, double* rel_res);

/* Evaporation rate of the current state, eqs. 17-21: total h^3 sum(mdot)
 * in kg/s, and optionally the volumetric source mdot (kg m^-3 s^-1) written
 * to a caller device cell array (NULL to skip).  In the literal species form
 * the liquid cells' omega and c are first set to their saturation values, as
 * at the start of a step (the gas cells and every other field are kept). */
int ds_evaporation_rate(ds_grid* g, double* kg_per_s, double* mdot_or_null, void* stream);

/* Liquid volume h^3 sum(alpha) of the current state [m^3]: the quantity
 * whose normalised equivalent diameter (d/d0)^2 with d = (6 V/pi)^(1/3) the
 * paper follows in time (Section 4, the d^2 law, and the comparisons of
 * Sections 5-6).  FP64 reduction in a fixed order.  Synchronises the stream. */
int ds_droplet_volume(ds_grid* g, double* m3, void* stream);

/* Diagnostics of the last step / solve (host struct, no device work): the
 * redistribution constant K of eq. 20, the total evaporation rate h^3
 * sum(mdot) of eqs. 17-19, droplet volume and fuel mass (liquid, eq. 4, plus
 * vapour, eq. 9) with the boundary outflows, and each linear solve's
 * iterations and residual (eqs. 7-9). */
int ds_get_diagnostics(const ds_grid* g, ds_diagnostics* out);

/* Internal fields of the last step, for parity tests: copies one array into
 * a caller device buffer of the stated size. */
enum {
  DS_FIELD_MDOT_RAW = 0,   /* cells: mdot before redistribution (eq. 17)     */
  DS_FIELD_MDOT = 1,       /* cells: mdot after redistribution (eq. 19)      */
  DS_FIELD_ALPHA1 = 2,     /* cells: alpha after the liquid source (eq. 4)   */
  DS_FIELD_C = 3,          /* cells: vapour partial density rho_G theta omega */
  DS_FIELD_USTAR = 4,      /* u faces of the momentum predictor              */
  DS_FIELD_VSTAR = 5,
  DS_FIELD_WSTAR = 6,
  DS_FIELD_ADJ = 7,        /* cells: flat index of adj (as double), -1 if none,
                              -2 off the interface                          */
  DS_FIELD_RHO_G = 8       /* cells: gas density of the state (eq. 24; the ambient value
                              everywhere with DS_GAS_AMBIENT)                  */
};
int ds_get_internal(ds_grid* g, int which, double* dst, size_t count, void* stream);

/* Measurement hook.  With timing enabled, HIP events on the caller's stream
 * bracket every launch of the pressure solve's fine-level conjugate-gradient
 * operator kernel (direction update p = z + beta p fused with the
 * matrix-free product q = A p and <p, q>) that performs an iteration;
 * ds_get_kernel_timing returns the mean duration in microseconds, the number
 * of timed launches and the kernel's algorithmic bytes per launch (each
 * array it streams counted once: z, p, q_coef read, and diag unless the
 * kernel forms it from q_coef, as it does for the multigrid-preconditioned
 * pressure-type systems; p, q written; on levels with nz a multiple of the
 * vector width also x read and written, the previous iteration's deferred
 * solution update).
 * Enabling resets the accumulators.  The event pool is created on first use
 * (host-side HIP objects, no device memory). */
int ds_set_kernel_timing(ds_grid* g, int enable);
int ds_get_kernel_timing(const ds_grid* g, double* avg_us, long long* launches, double* bytes_per_launch);

/* Measurement hook: replays the same operator kernel `reps` times back to
 * back on the current pressure system (the last one assembled by a step or
 * pressure solve, in the handle's precision) between two events on `stream`
 * and returns the mean duration (us) and the algorithmic bytes per launch.
 * Only solver scratch vectors are written; the state is untouched. */
int ds_time_operator_kernel(ds_grid* g, int reps, double* avg_us, double* bytes_per_launch, void* stream);

/* ---- Differentiation form: derivative of the liquid volume after a run.
 *
 * J = dJ_dV * V_N with V_N = h^3 sum(alpha) after nsteps steps (the droplet
 * volume whose evolution Section 4 follows).  The reverse sweep gives
 * dJ/d(D_v, dh_ev, T_amb) and dJ/d(initial alpha, T, omega, u, v, w).
 * Method: the exact derivative of the discrete step of Section 3.1 with its
 * integer decisions held (interface classes and adj of eqs. 15-17, donor and
 * limiter branches, inletOutlet switches, the clamps of the mixing rule of
 * eq. 31); linear solves (eqs. 7-9 and the liquid-transport potential)
 * differentiated implicitly with the same operators; Peng-Robinson
 * equilibrium (eqs. 22-25) by the implicit-function rule.  T_amb acts through
 * the gas density (eq. 24), the ambient boundary temperature and the inflow
 * face temperature; its effect through the initial temperature field is the
 * caller's (chain it with dJ/dT0).  The initial pressure only warm-starts the
 * first solve and carries no derivative.
 *
 * Memory: the tape is caller-owned device memory (256-byte aligned) of
 * ds_tape_bytes() bytes holding the adjoint arrays (about 36 arrays of the
 * grid, with the interface stage's per-cell records, which are summed per
 * target in a fixed order: the reverse sweep is bitwise reproducible) and the
 * stored states: a checkpoint every ckpt_every steps, the final
 * state, and ckpt_every-1 segment states recomputed during the reverse sweep
 * (about 10 arrays of the grid per stored state).  ckpt_every = 1 stores every
 * state and recomputes none; larger values trade one extra forward pass for
 * memory.  The tape must stay allocated and untouched between
 * ds_forward_record and ds_adjoint.  The library still allocates nothing. */

/* Tape size for nsteps steps with a checkpoint every ckpt_every steps
 * (0 on invalid arguments).  Host only. */
size_t ds_tape_bytes(const ds_grid* g, int nsteps, int ckpt_every);

/* Advance nsteps steps exactly as ds_step does, storing checkpoints in the
 * tape.  Returns ds_step's status (DS_ERR_NOT_CONVERGED if a solve hit
 * maxit).  DS_ERR_ARG for a small or misaligned tape, DS_ERR_STATE before
 * ds_set_fields.  Synchronises the stream at the end. */
int ds_forward_record(ds_grid* g, int nsteps, int ckpt_every, void* tape, size_t tape_bytes, void* stream);

/* Reverse sweep over the recorded run.  grads: host double[3] receiving
 * dJ/dD_v, dJ/ddh_ev, dJ/dT_amb.  dalpha0, dT0, domega0 (cell arrays) and
 * du0, dv0, dw0 (face arrays): device buffers receiving dJ/d(initial
 * field), each may be NULL.  Afterwards the handle holds the final state of
 * the run again (as after ds_forward_record).  DS_ERR_STATE without a
 * recorded run; DS_ERR_NOT_CONVERGED if an adjoint solve hit maxit (results
 * are still written); DS_ERR_NONFINITE for a non-finite gradient.  The
 * adjoint covers the conservative species form of the inviscid step:
 * ds_forward_record returns DS_ERR_ARG for a grid created with
 * DS_SPECIES_LITERAL or with viscous = 1.
 * Synchronises the stream. */
int ds_adjoint(ds_grid* g, double dJ_dV, double* grads, double* dalpha0, double* dT0, double* domega0,
               double* du0, double* dv0, double* dw0, void* stream);

/* Iterations of the adjoint linear solves of the last ds_adjoint, summed
 * over the steps: iters4[0] pressure, [1] species, [2] energy, [3] liquid-
 * transport potential.  Host only. */
int ds_get_adjoint_iterations(const ds_grid* g, int* iters4);

/* Measurement hook: replays one solver kernel `reps` times back to back on
 * the current pressure system (as ds_time_operator_kernel) and returns its
 * mean duration (us) and algorithmic bytes per launch.
 *   DS_KERNEL_CG_OPERATOR: the conjugate-gradient operator kernel (above);
 *   DS_KERNEL_MG_SMOOTH: one sweep of the multigrid preconditioner's
 *     smoother on the fine level, the kernel the V-cycle runs there: the
 *     coloured (x-z red-black) sweep where the level takes it, else damped
 *     Jacobi (reads r, x, q_coef and forms diag from q_coef; writes x: 4
 *     arrays either way).  Needs pressure_precond = 1.
 * Only solver scratch vectors are written.  DS_ERR_ARG for an unknown kernel. */
enum { DS_KERNEL_CG_OPERATOR = 0, DS_KERNEL_MG_SMOOTH = 1 };
int ds_time_kernel(ds_grid* g, int which, int reps, double* avg_us, double* bytes_per_launch, void* stream);

/* ---- For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 * Liquid volume h^3 sum(alpha) of a caller's device cell array alpha
 * (nx*ny*nz doubles, the layout above), written to the caller's device double
 * *m3: the quantity ds_droplet_volume returns for a handle whose state holds
 * the same alpha, bit for bit (same blocks, same fixed reduction order), with
 * no handle and no workspace.  Asynchronous on `stream` (no synchronisation;
 * the launches are kernels only, so the call can be captured into a graph).
 * The call allocates nothing: its only device memory beyond alpha and *m3 is
 * the library's own scratch, a file-scope device array of
 * DS_NOALLOC_SCRATCH_BYTES that every GPU the library runs on holds until the
 * process ends (block partials of the reduction and its completion counter,
 * which each call clears itself).  Calls that overlap on one GPU (two streams
 * or two host threads) share that array and race: serialise them.  Grids of
 * more than DS_NOALLOC_MAX_CELLS cells, extents below 1, h <= 0 and null
 * pointers return DS_ERR_ARG before anything is launched; the message is then
 * ds_last_error(NULL) on the calling thread. */
#define DS_NOALLOC_SCRATCH_BYTES 16640
#define DS_NOALLOC_MAX_CELLS 2147483647LL
int ds_droplet_volume_noalloc(const double* alpha, int nx, int ny, int nz, double h, double* m3, void* stream);

/* Message describing the last error on this handle ("" if none); with a NULL
 * handle, the calling thread's last failed handle-free call. */
const char* ds_last_error(const ds_grid* g);

#ifdef __cplusplus
}
#endif
#endif /* DSVOF_H */
