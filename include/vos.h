/*
 * vos.h -- C ABI of the MI355X (gfx950) Volume-of-Solid dissolution step.
 *
 * The library advances the micro-continuum model of Maes, Soulaine & Menke
 * ("Improved Volume-of-Solid formulations for micro-continuum simulation of
 * mineral dissolution at the pore-scale") on a uniform Cartesian voxel grid:
 * Darcy-Brinkman-Stokes momentum with Kozeny-Carman drag (Section 2.2,
 * Eq. momentumDBS, Eq. perm), the pressure equation from continuity
 * (Eq. contDBSQS), quasi-static advection-diffusion-reaction of the acid
 * (Eq. concentrationDBSQS) and the solid update (Eq. mbs) with the reaction
 * rate of iVoS (Eq. RfiVoS), VoS-psi or VoS-psi' (Eq. RfVoSpsi, Section 2.4).
 *
 * Conventions
 *  - Every call returns vos_status; VOS_OK is 0.  On failure the message of
 *    the calling thread is available from vos_last_error().  No C++
 *    exception crosses this boundary.
 *  - Units are SI with mol (the paper's kmol -> mol); p is the dynamic
 *    pressure in Pa.
 *  - Fields are FP64, x fastest: cell (i,j,k) at i + nx*(j + ny*k).  Face
 *    grids (MAC): x-faces (nx+1)*ny*nz, y-faces nx*(ny+1)*nz, z-faces
 *    nx*ny*(nz+1), indexed the same way over their own dims; face i of the
 *    x grid sits between cells i-1 and i.  nz == 1 is a 2-D problem (no z
 *    faces are used).
 *  - Boundaries: x = 0 inlet (plug velocity u_in, or with the pressure drive
 *    pressure p_in and zero normal gradient of u; concentration c_in),
 *    x = nx*dx outlet (pressure p_out, zero normal gradient of u and c),
 *    all other sides no-slip, no-flux walls.
 *  - Memory: the library never allocates device memory.  The caller sizes a
 *    workspace with vos_workspace_bytes(), allocates it (e.g. a torch
 *    tensor) and hands it to vos_create(); the library carves every device
 *    array from it.  The caller keeps ownership and must keep it alive until
 *    vos_destroy().  A small pinned host buffer is allocated for reading
 *    solver scalars back.
 *  - Streams: all work is enqueued on the hipStream_t given to vos_create().
 *    Calls on one handle are not thread-safe; different handles are
 *    independent.  Every call that returns data to the host synchronises
 *    that stream.
 */
#ifndef VOS_H
#define VOS_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VOS_OK = 0,
  VOS_ERR_ARG = 1,     /* invalid argument (sizes, pointers, parameter ranges) */
  VOS_ERR_DEVICE = 2,  /* a HIP runtime call failed */
  VOS_ERR_NOCONV = 3,  /* a Krylov solve hit its iteration cap */
  VOS_ERR_OOM = 4,     /* the workspace is smaller than vos_workspace_bytes() */
  VOS_ERR_STATE = 5    /* call out of order (e.g. a step before the geometry) */
} vos_status;

/* Uniform voxel grid: nx >= 2, ny >= 1, nz >= 1 cells of edge dx [m]. */
typedef struct { int nx, ny, nz; double dx; } vos_grid;

/* Reaction-rate closure (Section 2.3 / 2.4). */
typedef enum {
  VOS_IVOS = 0,        /* Eq. RfiVoS: divergence of the reactive flux */
  VOS_PSI = 1,         /* Eq. RfVoSpsi with psi = 4 eps (1 - eps) */
  VOS_PSI_PRIME = 2    /* psi = lambda(eps) eps (1 - eps), lambda refitted every step */
} vos_model;

/* Arithmetic of the multigrid preconditioners. */
typedef enum {
  VOS_FP64 = 0,        /* everything FP64 */
  VOS_MIXED = 1        /* FP32 multigrid (smoothing, restriction, prolongation)
                          for the pressure and momentum systems inside FP64 CG:
                          residuals, dot products, right-hand sides and every
                          global balance stay FP64.  The transport hierarchy is
                          FP64 in both modes (its coarse operators of
                          upwind-dominated rows lose their diagonal in FP32) */
} vos_precision;

/* Physical parameters (Tables 1-3 of the paper give realistic values). */
typedef struct {
  double mu;        /* dynamic viscosity [Pa s] */
  double rho;       /* fluid density [kg/m3] */
  double D;         /* molecular diffusion coefficient [m2/s]; D* = D */
  double k0;        /* Kozeny-Carman constant [m2] (Eq. perm) */
  double kc;        /* surface reaction constant [m/s], R = kc c */
  double Vm;        /* M_ws / rho_s [m3/mol] (Eq. mbs) */
  double zeta;      /* stoichiometric coefficient of the acid */
  double c_in;      /* inlet concentration [mol/m3] */
  double eps_min;   /* porosity floor of the solid (Appendix C uses 1e-4) */
  double u_in;      /* inlet plug velocity [m/s], >= 0 (drive 0) */
  double p_out;     /* outlet pressure [Pa] */
  int model;        /* vos_model */
  int drive;        /* 0: inlet plug velocity u_in; 1: inlet pressure p_in (Section 3.3 drives its
                       micro-CT sample at constant pressure); the inlet faces then are unknowns */
  double p_in;      /* inlet pressure [Pa] (drive 1) */
  int convection;   /* 1: explicit first-order upwind momentum convection, the u u / eps term of
                       Eq. momentumDBS (0: creeping flow without it) */
  int grad_scheme;  /* 0: central gradient of eps; 1: decentred (Section 2.4: per direction the
                       one-sided difference toward the neighbour of larger eps); VoS-psi only */
  int psi_kind;     /* 0: psi = lambda eps (1 - eps); 1: psi = 1, i.e. a_s = |grad eps| (Section 2.4);
                       psi = 1 is for VOS_PSI (lambda is fitted to eps (1 - eps)) */
  int transient;    /* 1: the transient terms of Section 2.2 -- storage d(eps c)/dt in the transport
                       equation (Eq. concentrationDBS) and the dissolution source
                       Rbar (Vm - Vm_f) of Eq. contDBS (lagged rates) in the continuity equation */
  double Vm_f;      /* M_ws / rho of the fluid [m3/mol] (the source's second term), >= 0 */
} vos_params;

/* Solver options.  Tolerances are relative Jacobi-scaled residual norms:
 * momentum and pressure ||D^-1/2 r|| <= rtol ||D^-1/2 b||, transport
 * ||D^-1 r|| <= rtol ||D^-1 b|| (D the matrix diagonal). */
typedef struct {
  double rtol_u, rtol_p, rtol_c;
  int maxit_u, maxit_p, maxit_c;
  int precision;    /* vos_precision (pressure multigrid) */
  int mg_nu;        /* Jacobi sweeps before and after each coarse correction of the pressure
                       and momentum hierarchies, 1..8; 0: pressure 4 in 2-D and 3 in 3-D,
                       momentum 2.  The transport hierarchy uses at most 2. */
  int check_every;  /* Krylov iterations launched between host convergence checks, 1..256; the
                       first check of a solve comes after as many such chunks as fit in the
                       iterations the previous solve of the same system took */
  int use_graphs;   /* 1: capture each solve's chunk of check_every iterations in a HIP graph
                       once and replay it (iteration counts then round up to a multiple of
                       check_every in the worst case; results are identical); 0: plain launches.
                       Ignored (off) when vos_create() is given the null stream. */
  int coarse_cells; /* multigrid levels with at most this many cells run inside one single-block
                       kernel, 64..65536 (0: 2048) */
  int level_kernels;/* kernels of the fine multigrid levels: 0 fused (2-D: one tiled kernel per
                       leg of a level; 3-D: sweeps that march through z with the neighbours in
                       LDS and registers); 1 one plain kernel per sweep.  Both form every value
                       by the same expression: results are bitwise identical. */
  int p_fp32_its;   /* VOS_MIXED: at most this many pressure iterations per solve with the FP32
                       hierarchy before the solve continues with an FP64 one (0: no limit).
                       Independently, a solve switches once its residual has not halved within
                       400 iterations (FP32 rounding can stall the outer CG above 1e-8 when the
                       diagonal spans many orders of magnitude), and the later solves then use
                       the FP64 hierarchy from the start until the next
                       vos_set_solid_fraction.  >= 0. */
  int extrapolate;  /* 1: the pressure and transport solves start from the linear extrapolation
                       2 x^n - x^(n-1) of the last two steps' solutions, the momentum predictor
                       from 2 u*^n - u*^(n-1) of the last two predictors (x^n, or u^n, until
                       that history exists again after vos_create, vos_set_field,
                       vos_set_solid_fraction or vos_set_params; the pressure keeps p^n while
                       a warm-start network is attached); right-hand sides are unchanged.
                       2: as 1, but a solve starts from the quadratic extrapolation
                       3 x^n - 3 x^(n-1) + x^(n-2) whenever, at its previous start, the
                       quadratic prediction of x^n from the three solutions before it was
                       closer to x^n than the linear one (decided on the device).
                       0: start from x^n (u^n). */
  int setup_every;  /* the momentum and pressure multigrid hierarchies (coarse operators and
                       coarsest inverses) are rebuilt every this many steps and after every
                       state change
                       (vos_set_solid_fraction, vos_set_params, vos_set_field, a new time step
                       size); in between, a solve is preconditioned with the hierarchy of an
                       earlier step.  The Krylov iteration always applies the current operator,
                       so every solve still meets its tolerance.  The transport hierarchy is
                       rebuilt every step.  0 or 1: every step; <= 1000. */
  double deps_max;  /* Appendix D's bound on the change of eps per step: > 0 shortens the solid
                       update of a step to dt_s = min(dt, deps_max / max |Vm Rbar|), the maximum
                       over the cells whose distance to the clip bound in the direction of their
                       change exceeds deps_max, with Rbar the rates just computed (the flow and
                       transport solves keep dt); vos_diag.dt_solid reports dt_s.  0: dt_s = dt.
                       Finite, >= 0. */
  int simple;       /* 1: the quasi-static SIMPLE loop of Appendices A and B instead of one pass:
                       with eps frozen, steady momentum (Eq. momentumDBSQS, no inertia) under
                       implicit relaxation relax_u, the SIMPLE pressure correction, explicit
                       pressure relaxation relax_p, transport (implicit relaxation relax_c),
                       reaction rate -- repeated until the initial relative residual of every
                       solve is <= outer_tol (or outer_max times), then the solid update.  dt
                       then only caps the solid step (with deps_max: adaptive time stepping,
                       Appendix D).  Not with extrapolate != 0. */
  int outer_max;    /* SIMPLE: most outer iterations per step, >= 1 */
  double outer_tol; /* SIMPLE: convergence tolerance on the solves' initial residuals, >= 0 */
  double relax_u, relax_p, relax_c;  /* SIMPLE under-relaxation factors in (0, 1] (the paper: 0.3) */
  double solid_dt;  /* > 0: the solid update's own nominal step (before the deps_max bound), dt
                       then serving the flow alone, as the pseudo time step of its backward-Euler
                       inertia (Appendix A's quasi-static reading: flow and transport are steady,
                       the solid interface alone sets the physical step).  0: the solid advances
                       by dt.  Finite, >= 0; not with params->transient (its storage terms take
                       dt). */
} vos_opts;

/* Per-step diagnostics (Section 2.5 and Section 3.3 quantities, balances). */
typedef struct {
  int it_u[3], it_p, it_c;       /* Krylov iterations of the last step */
  double res_u[3], res_p, res_c; /* final relative residuals (see vos_opts) */
  double lambda;                 /* psi prefactor used (4 for iVoS / VoS-psi) */
  double solid_volume;           /* sum (1 - eps) V after the update       [m3] */
  double surface_area;           /* sum |grad eps| V at the step's start    [m2] */
  double porosity;               /* mean eps after the update */
  double dP;                     /* mean inlet-cell p - p_out (drive 1: p_in - p_out) [Pa] */
  double K;                      /* mu U_D L_D / dP (Section 2.5); L_D = (nx - 1/2) dx from the
                                    inlet cells (drive 0) or nx dx (drive 1)  [m2] */
  double acid_in, acid_out;      /* inlet / outlet acid flux            [mol/s] */
  double acid_consumed;          /* zeta * sum of the acid sink         [mol/s] */
  double solid_rate;             /* sum Rbar V                          [mol/s] */
  double acid_balance_rel;       /* (in - out - consumed - storage) / in */
  double solid_balance_rel;      /* (sum d(eps)V - dt Vm sum Rbar V + clipped) / (dt Vm |sum Rbar V|) */
  double clipped_volume;         /* sum (eps_unclipped - eps_clipped) V    [m3] */
  double max_deps;               /* max |eps^{n+1} - eps^n| */
  double alpha;                  /* (1/a) sum c|grad eps|V / sum eps c V (Section 2.5) */
  double t_ms[6];                /* GPU time of coefficients, momentum, pressure,
                                    correction, transport, reaction+update [ms] */
  int guess;                     /* pressure start: -1 p^n (no network attached),
                                    0 p^n (network guess rejected or off), 1 network guess */
  double res0_prev, res0_guess;  /* with a network attached: relative Jacobi-scaled residual
                                    of p^n and of the network guess (0 when off) */
  double guess_error_drop;       /* with the guess on: the fraction of the squared A-norm error
                                    of starting from p^n that the guess removed, in [0, 1],
                                    measured against the converged solution */
  int it_p_fp64;                 /* VOS_MIXED: pressure iterations run with the FP64 hierarchy
                                    after the FP32 one stalled or reached p_fp32_its (0: none) */
  double dt_solid;               /* time step of the solid update (dt unless vos_opts.deps_max
                                    shortened it)                          [s] */
  double U_D;                    /* Darcy velocity Q_in / A_in (Section 2.5)  [m/s] */
  double R_omega;                /* Section 3.3's macroscopic rate: porosity change / (Vm dt_s)
                                                                         [mol/m3/s] */
  double acid_accum;             /* transient storage sum (eps c - eps_prev c0) V / dt [mol/s] */
  int outer_its;                 /* outer iterations of the step (1 for one pass) */
  double outer_res;              /* largest initial relative residual of the last outer iteration */
  double div_source;             /* continuity source summed over the cells     [m3/s] */
} vos_diag;

/* Fields for vos_set_field / vos_get_field / vos_field_ptr. */
typedef enum {
  VOS_FIELD_EPS = 0,     /* porosity eps (cells) */
  VOS_FIELD_UX = 1,      /* face velocities (x, y, z face grids) */
  VOS_FIELD_UY = 2,
  VOS_FIELD_UZ = 3,
  VOS_FIELD_P = 4,       /* pressure (cells) */
  VOS_FIELD_C = 5,       /* acid concentration (cells) */
  VOS_FIELD_USTAR_X = 6, /* last momentum predictor (face grids; read only) */
  VOS_FIELD_USTAR_Y = 7,
  VOS_FIELD_USTAR_Z = 8,
  VOS_FIELD_RBAR = 9,    /* last reaction rate Rbar [mol/m3/s] (cells; read only) */
  VOS_FIELD_GMAG = 10,   /* |grad eps| of the last step's start (cells; read only) */
  VOS_FIELD_PDIAG = 11   /* diagonal of the last step's pressure matrix (cells; read only) */
} vos_field;

typedef struct vos_sim vos_sim;

/* Bytes of device workspace a simulation of this grid and options needs. */
vos_status vos_workspace_bytes(const vos_grid *grid, const vos_opts *opts, size_t *bytes);

/* Create a simulation.  workspace: device pointer of at least
 * vos_workspace_bytes() bytes, 256-byte aligned, owned by the caller.
 * hip_stream: a hipStream_t (NULL = the null stream).  The state starts
 * as fluid everywhere at rest with p = p_out and c = 0. */
vos_status vos_create(const vos_grid *grid, const vos_params *params, const vos_opts *opts,
                      void *workspace, size_t workspace_bytes, void *hip_stream, vos_sim **out);

vos_status vos_destroy(vos_sim *sim);

/* Geometry from the solid fraction eps_s in [0,1] (one value per cell):
 * eps = clamp(1 - eps_s, eps_min, 1) (Appendix C).  Also resets the inlet
 * face velocities to u_in.  eps_s is a host pointer (on_device = 0) or a
 * device pointer (on_device = 1).  Values outside [0,1] give VOS_ERR_ARG. */
vos_status vos_set_solid_fraction(vos_sim *sim, const double *eps_s, int on_device);

/* Replace the physical parameters (same grid and workspace).  The fields are
 * kept, except the inlet faces, which take the new u_in.  Used e.g. to set
 * the inlet velocity and kc for a target Peclet / Damkohler number once the
 * permeability of the geometry is known (Section 3.2). */
vos_status vos_set_params(vos_sim *sim, const vos_params *params);

/* Copy a whole field in or out (host or device buffer of the field's size).
 * Read-only fields reject vos_set_field with VOS_ERR_ARG. */
vos_status vos_set_field(vos_sim *sim, int field, const double *src, int on_device);
vos_status vos_get_field(vos_sim *sim, int field, double *dst, int on_device);

/* Borrowed device pointer of a field, valid until vos_destroy(). */
vos_status vos_field_ptr(vos_sim *sim, int field, double **dev_ptr);

/* Advance nsteps time steps of size dt [s].  Each step: coefficients from
 * eps^n, momentum predictor, pressure equation (multigrid-preconditioned CG),
 * velocity correction, quasi-static transport (BiCGStab), reaction rate and
 * solid update.  flags bit 0 (VOS_FREEZE_SOLID): skip the solid update (flow
 * and transport only; used to relax the initial state).  last (may be NULL)
 * receives the diagnostics of the final step.  A solve that reaches its
 * iteration cap stops the call with VOS_ERR_NOCONV after that step's update
 * (the diagnostics say which solve). */
#define VOS_FREEZE_SOLID 1
vos_status vos_step(vos_sim *sim, double dt, int nsteps, int flags, vos_diag *last);

/* Diagnostics of the current state without advancing it (iteration counts
 * and balances are those of the last step). */
vos_status vos_diagnostics(vos_sim *sim, vos_diag *out);

/* The pressure equation alone (stage S3; Eq. contDBSQS combined with the
 * momentum equation, Appendix B): coefficients from the current eps for a
 * step of dt [s] (the transmissibilities depend on it), right-hand side
 * -div(u) + A p from the current face velocities taken as the predictor u*
 * and the current p (plus the continuity source when transient), solved by
 * the multigrid-preconditioned flexible CG to opts.rtol_p.  Starts from guess
 * (nx*ny*nz doubles, device pointer if on_device, else host; NULL: the
 * current p) and leaves the solution in the P field.  Velocities are not
 * corrected; eps is not changed.  out (may be NULL) receives it_p, res_p,
 * it_p_fp64 and t_ms[2].  VOS_ERR_NOCONV if the cap is reached (p then holds
 * the last iterate). */
vos_status vos_solve_pressure(vos_sim *sim, double dt, const double *guess, int on_device, vos_diag *out);

/* The set-up of a run from a geometry (not timed): with eps frozen, repeat
 * the flow stages (coefficients, momentum predictor, pressure, correction)
 * with steps of dt until the relative change of the face velocities over an
 * iteration, ||u - u_prev|| / ||u||, is <= tol (at most max_iters times), then
 * the concentration: one transport solve with pure upwind convection, then one
 * with the van Leer correction lagged on that result.  out (may be NULL):
 * outer_its (flow iterations), outer_res (the last relative change), the
 * solves' counts.  VOS_ERR_NOCONV if the flow has not settled within
 * max_iters (the state is then the last iterate, c^0 included). */
vos_status vos_initialize(vos_sim *sim, double dt, int max_iters, double tol, vos_diag *out);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): the pressure equation of
 * vos_solve_pressure for a state the caller passes in, with no simulation
 * handle and no workspace.  All inputs and outputs are device pointers on the
 * current device: eps (cells), the face velocities ux, uy, uz (taken as the
 * predictor u*; uz may be NULL in 2-D) and p (cells: the current pressure on
 * entry, the solution on exit).  Every scratch buffer comes from one static
 * device array of 48 MiB per GPU (held until the process ends), enough for
 * about 2.0e5 cells in 2-D (512 x 384) and 2.4e5 in 3-D (62^3); larger grids
 * give VOS_ERR_ARG with the bytes they would need.  Plain launches on hip_stream, no graph
 * capture, no hipMalloc / hipFree or other allocating call.  Calls on one GPU
 * share the array (and, in one process, a host control block): calls that
 * overlap race, so serialise them.  params->transient must be 0 (no lagged
 * rates for the continuity source).  out as for vos_solve_pressure. */
vos_status vos_solve_pressure_noalloc(const vos_grid *grid, const vos_params *params, const vos_opts *opts,
                                      double dt, const double *eps, const double *ux, const double *uy,
                                      const double *uz, double *p, void *hip_stream, vos_diag *out);

/* Checkpoint of the physical state: eps, the face velocities, p, c and the
 * two arrays the transient terms carry between steps (eps at the previous
 * step's start, the previous rates), with a header naming the grid.
 * vos_state_bytes gives the size of that host buffer; vos_get_state fills it
 * (bytes must be at least that size); vos_set_state restores it into a
 * simulation of the same grid (VOS_ERR_ARG on a size, grid or format
 * mismatch).  After a restore every solve starts from the restored state and
 * rebuilds its hierarchies, so the run continues bitwise as it would have
 * when extrapolate = 0 and setup_every <= 1, and within the solvers'
 * tolerances otherwise (extrapolation histories are not part of the state). */
vos_status vos_state_bytes(vos_sim *sim, size_t *bytes);
vos_status vos_get_state(vos_sim *sim, void *buf, size_t bytes);
vos_status vos_set_state(vos_sim *sim, const void *buf, size_t bytes);

/* Kernel families for vos_time_kernel. */
typedef enum {
  VOS_KERNEL_V_RESTRICT = 0,  /* residual restriction, every fine level of the transport hierarchy */
  VOS_KERNEL_V_POST = 1,      /* prolongation + first post-smoothing sweep, same levels */
  VOS_KERNEL_V_PRE = 2,       /* first two pre-smoothing sweeps, same levels */
  VOS_KERNEL_V_COARSE = 3,    /* the single-block coarse tail of the transport V-cycle (in LDS in 2-D) */
  VOS_KERNEL_P_APPLY = 4,     /* pressure operator application (FP64) */
  VOS_KERNEL_ADR_APPLY = 5,   /* transport operator application (FP64) */
  VOS_KERNEL_V_DOWN = 6,      /* 2-D tiled down leg (pre-sweeps + restriction), finest transport level */
  VOS_KERNEL_V_UP = 7,        /* 2-D tiled up leg (prolongation + post-sweeps), finest transport level */
  /* 3-D pressure hierarchy, finest level, z-marching kernels in the arithmetic of the
     hierarchy the last pressure solve used (FP32 in mixed precision unless it fell back): */
  VOS_KERNEL_P_PRE3D = 8,     /* first down launch: two damped-Jacobi sweeps from the FP64 residual */
  VOS_KERNEL_P_SWEEP3D = 9,   /* one further damped-Jacobi sweep */
  VOS_KERNEL_P_RESTRICT3D = 10, /* residual restricted to the next level */
  VOS_KERNEL_P_POST3D = 11,   /* prolongation fused with the first up sweep */
  /* the same four kernels on the finest level of the 3-D transport hierarchy (FP64): */
  VOS_KERNEL_C_PRE3D = 12,
  VOS_KERNEL_C_SWEEP3D = 13,
  VOS_KERNEL_C_RESTRICT3D = 14,
  VOS_KERNEL_C_POST3D = 15,
  /* the fused legs of that level (levels of >= 2^20 cells): both pre-sweeps and the
     restriction; the prolongation and both post-sweeps with the FP64 output */
  VOS_KERNEL_C_DOWN3D = 16,
  VOS_KERNEL_C_UP3D = 17,
  /* the same two fused legs on the finest level of the x-momentum hierarchy (the
     (nx+1) x ny x nz face grid; FP32 in mixed precision, else FP64): */
  VOS_KERNEL_M_DOWN3D = 18,
  VOS_KERNEL_M_UP3D = 19
} vos_kernel_family;

/* Time `reps` back-to-back launch sequences of one kernel family on the live
 * state (after at least one vos_step), between two HIP events on the
 * simulation's stream.  A sequence is one launch per level for the V-cycle
 * families, else one launch.  Outputs: average duration of one launch [ms]
 * and its algorithmic bytes (every array read or written once per launch,
 * neighbour re-reads not counted).  The kernels write only scratch buffers. */
vos_status vos_time_kernel(vos_sim *sim, int family, int reps, double *avg_launch_ms, double *bytes_per_launch);

/* Thread-local message of the last failed call on this thread ("" if none). */
const char *vos_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* VOS_H */
