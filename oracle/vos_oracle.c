/*
 * vos_oracle.c -- plain, slow FP64 CPU oracle of one Volume-of-Solid time step
 * (Maes, Soulaine & Menke, "Improved Volume-of-Solid formulations for
 * micro-continuum simulation of mineral dissolution at the pore-scale").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark load it (through oracle/__init__.py).  It shares no code,
 * header or constant with the HIP path.
 *
 * Everything is written as direct loops over cells and faces, in the order the
 * step is defined, with no blocking or fusion.  Linear systems are assembled as
 * explicit 7-point stencils and solved with textbook Jacobi-preconditioned CG
 * (symmetric systems) or BiCGStab (van der Vorst 1992, on the row-scaled
 * non-symmetric transport system).
 *
 * Step (one pass, the reading of the paper's solution procedure, Appendix B):
 *  S1 coefficients from eps^n: face porosity (Gauss linear interpolation),
 *     Kozeny-Carman drag (Eq. perm, Eq. momentumDBS), momentum diagonal,
 *     pressure transmissibility, grad(eps), interface normal n_s = -grad/|grad|
 *     (Section 2.3), reactive face velocity w_f = k_c n_f . S_f, and the
 *     localization function psi = lambda eps (1-eps) (Section 2.4).
 *  S2 momentum predictor: backward-Euler Darcy-Brinkman-Stokes (Eq. momentumDBS)
 *     row-scaled by eps_f, with the old pressure gradient.
 *  S3 pressure equation from continuity (Eq. contDBSQS) and momentum (SIMPLE).
 *  S4 face-velocity correction.
 *  S5 quasi-static advection-diffusion-reaction (Eq. concentrationDBSQS) with
 *     van Leer (1974) convection by deferred correction on c^n.
 *  S6 reaction rate: iVoS (Eq. RfiVoS) or VoS-psi / VoS-psi' (Eq. RfVoSpsi),
 *     then the solid balance (Eq. mbs) with eps clipped to [eps_min, 1].
 *  S7 FP64 diagnostics (Section 2.5 upscaled quantities, balances).
 *
 * Options beyond that single pass (all off by default):
 *  - inlet pressure drive (Section 3.3 drives Benchmark 3 at constant pressure);
 *  - explicit first-order upwind momentum convection (the u u / eps term of
 *    Eq. momentumDBS);
 *  - the quasi-static SIMPLE outer loop of Appendices A and B: steady momentum
 *    (Eq. momentumDBSQS) with implicit under-relaxation, explicit pressure
 *    relaxation, transport and reaction rate every outer iteration, repeated
 *    until the initial residuals of the solves fall below a tolerance;
 *  - the transient terms of Section 2.2: storage d(eps c)/dt in the transport
 *    equation (Eq. concentrationDBS) and the dissolution source of
 *    Eq. contDBS in the continuity equation;
 *  - the VoS-psi variants of Section 2.4: a decentred gradient and psi = 1.
 *
 * Parity pinned by tests/test_oracle_*.py against closed forms, brute-force
 * dense solves and the paper's worked numbers.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ types */

typedef struct {
  int nx, ny, nz;          /* cells; nz == 1 means a 2-D problem */
  double dx;               /* voxel edge [m] */
  double mu, rho;          /* dynamic viscosity [Pa s], density [kg/m3] */
  double D;                /* molecular diffusion [m2/s] (D* = D) */
  double k0;               /* Kozeny-Carman constant [m2] */
  double kc;               /* surface reaction constant [m/s] */
  double Vm;               /* M_ws / rho_s [m3/mol] */
  double zeta;             /* stoichiometric coefficient of the acid */
  double c_in;             /* inlet concentration [mol/m3] */
  double eps_min;          /* porosity floor in the solid */
  double u_in;             /* inlet (plug) velocity [m/s] */
  double p_out;            /* outlet pressure [Pa] */
  int model;               /* 0 iVoS, 1 VoS-psi (lambda = 4), 2 VoS-psi' */
  double rtol_u, rtol_p, rtol_c;
  int maxit_u, maxit_p, maxit_c;
  double deps_max;         /* > 0: the solid update's step is shortened so that no cell's
                              eps changes by more than this (Appendix D); 0: dt */
  int drive;               /* 0: inlet plug velocity u_in; 1: inlet pressure p_in (the inlet
                              faces are then unknowns, like the outlet's) */
  double p_in;             /* inlet pressure [Pa] (drive 1) */
  int convection;          /* 1: explicit first-order upwind momentum convection */
  int grad_scheme;         /* 0: central gradient of eps; 1: decentred (VoS-psi variants) */
  int psi_kind;            /* 0: psi = lambda eps (1 - eps); 1: psi = 1 (a_s = |grad eps|) */
  int transient;           /* 1: storage d(eps c)/dt and the continuity source of Eq. contDBS */
  double Vm_f;             /* M_ws / rho of the fluid [m3/mol] (continuity source) */
  int simple;              /* 1: quasi-static SIMPLE outer loop (Appendices A, B) */
  int outer_max;           /* SIMPLE: most outer iterations per step */
  double outer_tol;        /* SIMPLE: stop once every solve's initial residual is <= this */
  double relax_u, relax_p, relax_c;   /* SIMPLE under-relaxation factors in (0, 1] */
  double solid_dt;         /* > 0: the solid update's own step (before the deps_max bound),
                              dt then serving the flow alone as its pseudo time step;
                              0: the solid advances by dt */
} orc_prob;

typedef struct {
  int it_u[3], it_p, it_c;
  double res_u[3], res_p, res_c;       /* final Jacobi-scaled relative residuals */
  double lambda;                       /* psi prefactor used this step */
  double solid_volume;                 /* sum (1-eps^{n+1}) V                 [m3] */
  double surface_area;                 /* sum |grad eps^n| V                  [m2] */
  double porosity;                     /* mean eps^{n+1} */
  double dP;                           /* mean inlet-cell p - p_out           [Pa] */
  double K;                            /* mu U_D L_D / dP                     [m2] */
  double acid_in, acid_out;            /* inlet / outlet acid fluxes      [mol/s] */
  double acid_consumed;                /* zeta * sum of the acid sink     [mol/s] */
  double solid_rate;                   /* sum Rbar V                      [mol/s] */
  double acid_balance_rel;             /* (in - out - consumed) / in */
  double solid_balance_rel;            /* (sum dEps V - dt Vm sum Rbar V + clip) / (dt Vm |sum Rbar V|) */
  double clipped_volume;               /* sum (eps_unclipped - eps_clipped) V  [m3] */
  double max_deps;                     /* max |eps^{n+1} - eps^n| */
  double alpha;                        /* (1/a) sum c|g|V / sum eps c V */
  double dt_solid;                     /* time step of the solid update        [s] */
  double U_D;                          /* Darcy velocity Q_in / A_in            [m/s] */
  double R_omega;                      /* Section 3.3: d(porosity) / (V_m dt_s)  [mol/m3/s] */
  double acid_accum;                   /* transient storage sum (eps c)' V / dt [mol/s] */
  int outer_its;                       /* SIMPLE outer iterations taken (1 for one pass) */
  double outer_res;                    /* largest initial relative residual of the last outer iteration */
  double div_source;                   /* sum of the continuity source over the cells [m3/s] */
} orc_diag;

/* Optional intermediate outputs of a step (any pointer may be NULL). */
typedef struct {
  double *ustar[3];        /* momentum predictor on the three face grids */
  double *rbar;            /* solid reaction rate [mol/m3/s] per cell */
  double *sink;            /* acid sink per cell [mol/s] (before zeta) */
  double *gmag;            /* |grad eps^n| per cell */
} orc_out;

/* State carried between steps besides the fields (may be NULL when the
 * transient terms are off): eps at the start of the previous step (the
 * storage term's eps^{n-1}) and the previous step's reaction rate (the lagged
 * continuity source).  Both are read, then overwritten for the next step. */
typedef struct {
  double *eps_prev;
  double *rbar_prev;
} orc_aux;

enum { ORC_OK = 0, ORC_ERR_ARG = 1, ORC_ERR_NOCONV = 3, ORC_ERR_OOM = 4 };

/* ------------------------------------------------------------- the grid */

typedef struct {
  int n[3];
  int nd;
  int drive;               /* 1: the inlet faces are momentum unknowns (pressure drive) */
  double dx, S, V;
  long nc;
  long nf[3];
  int fd[3][3];            /* face-grid dims: fd[d][e] = n[e] + (e == d) */
} grid_t;

static void grid_init(grid_t *g, const orc_prob *P)
{
  g->n[0] = P->nx; g->n[1] = P->ny; g->n[2] = P->nz;
  g->nd = (P->nz == 1) ? 2 : 3;
  g->drive = P->drive;
  g->dx = P->dx; g->S = P->dx * P->dx; g->V = g->S * P->dx;
  g->nc = (long)P->nx * P->ny * P->nz;
  for (int d = 0; d < 3; ++d) {
    for (int e = 0; e < 3; ++e) g->fd[d][e] = g->n[e] + (e == d);
    g->nf[d] = (long)g->fd[d][0] * g->fd[d][1] * g->fd[d][2];
  }
}

static long cidx(const grid_t *g, const int x[3])
{
  return x[0] + (long)g->n[0] * (x[1] + (long)g->n[1] * x[2]);
}

/* Face (d, x) separates cell x - e_d (lower) from cell x (upper); x[d] in [0, n[d]]. */
static long fidx(const grid_t *g, int d, const int x[3])
{
  return x[0] + (long)g->fd[d][0] * (x[1] + (long)g->fd[d][1] * x[2]);
}

static void unflatten(const int dims[3], long id, int x[3])
{
  x[0] = (int)(id % dims[0]); id /= dims[0];
  x[1] = (int)(id % dims[1]); x[2] = (int)(id / dims[1]);
}

enum { F_INTERIOR, F_INLET, F_OUTLET, F_WALL };

static int face_kind(const grid_t *g, int d, int q)
{
  if (q > 0 && q < g->n[d]) return F_INTERIOR;
  if (d == 0) return q == 0 ? F_INLET : F_OUTLET;
  return F_WALL;
}

/* A momentum unknown: interior faces, plus the outlet faces of the x grid,
 * plus its inlet faces under a pressure drive. */
static int mom_unknown(const grid_t *g, int d, const int x[3])
{
  int k = face_kind(g, d, x[d]);
  return k == F_INTERIOR || k == F_OUTLET || (k == F_INLET && g->drive);
}

/* ----------------------------------------------- 7-point stencil systems */

/* a[0] centre, a[1] -x, a[2] +x, a[3] -y, a[4] +y, a[5] -z, a[6] +z; each an
 * array over the grid of dims n.  An entry pointing outside the grid is 0. */
typedef struct {
  int n[3];
  long N;
  double *a[7];
} stencil_t;

static int stencil_alloc(stencil_t *A, const int n[3])
{
  A->n[0] = n[0]; A->n[1] = n[1]; A->n[2] = n[2];
  A->N = (long)n[0] * n[1] * n[2];
  for (int k = 0; k < 7; ++k) {
    A->a[k] = (double *)calloc((size_t)A->N, sizeof(double));
    if (!A->a[k]) return ORC_ERR_OOM;
  }
  return ORC_OK;
}

static void stencil_free(stencil_t *A)
{
  for (int k = 0; k < 7; ++k) { free(A->a[k]); A->a[k] = NULL; }
}

static void stencil_apply(const stencil_t *A, const double *x, double *y)
{
  const long sx = 1, sy = A->n[0], sz = (long)A->n[0] * A->n[1];
  for (long id = 0; id < A->N; ++id) {
    int c[3];
    unflatten(A->n, id, c);
    double v = A->a[0][id] * x[id];
    if (c[0] > 0)           v += A->a[1][id] * x[id - sx];
    if (c[0] < A->n[0] - 1) v += A->a[2][id] * x[id + sx];
    if (c[1] > 0)           v += A->a[3][id] * x[id - sy];
    if (c[1] < A->n[1] - 1) v += A->a[4][id] * x[id + sy];
    if (c[2] > 0)           v += A->a[5][id] * x[id - sz];
    if (c[2] < A->n[2] - 1) v += A->a[6][id] * x[id + sz];
    y[id] = v;
  }
}

static double dot(long n, const double *a, const double *b)
{
  double s = 0.0;
  for (long i = 0; i < n; ++i) s += a[i] * b[i];
  return s;
}

/* Jacobi-preconditioned CG.  Stops when ||D^{-1/2} r|| <= rtol ||D^{-1/2} b||
 * (for M = D, r.z is exactly that squared norm). */
static int pcg_jacobi(const stencil_t *A, const double *b, double *x, double rtol,
                      int maxit, int *its, double *relres, double *relres0)
{
  long N = A->N;
  double *r = malloc(N * sizeof(double)), *z = malloc(N * sizeof(double));
  double *p = malloc(N * sizeof(double)), *q = malloc(N * sizeof(double));
  if (!r || !z || !p || !q) { free(r); free(z); free(p); free(q); return ORC_ERR_OOM; }
  double bnorm2 = 0.0;
  for (long i = 0; i < N; ++i) bnorm2 += b[i] * b[i] / A->a[0][i];
  stencil_apply(A, x, q);
  for (long i = 0; i < N; ++i) { r[i] = b[i] - q[i]; z[i] = r[i] / A->a[0][i]; p[i] = z[i]; }
  double rz = dot(N, r, z);
  if (relres0) *relres0 = bnorm2 > 0.0 ? sqrt(rz / bnorm2) : 0.0;
  int k = 0, status = ORC_ERR_NOCONV;
  double tol2 = rtol * rtol * bnorm2;
  while (1) {
    if (rz <= tol2 || rz == 0.0) { status = ORC_OK; break; }
    if (k >= maxit) break;
    stencil_apply(A, p, q);
    double alpha = rz / dot(N, p, q);
    for (long i = 0; i < N; ++i) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; z[i] = r[i] / A->a[0][i]; }
    double rz_new = dot(N, r, z);
    double beta = rz_new / rz;
    rz = rz_new;
    for (long i = 0; i < N; ++i) p[i] = z[i] + beta * p[i];
    ++k;
  }
  *its = k;
  *relres = bnorm2 > 0.0 ? sqrt(rz / bnorm2) : 0.0;
  free(r); free(z); free(p); free(q);
  return status;
}

/* splitmix64 (Steele, Lea & Flood 2014): the 64-bit output of counter i,
 * mapped to a double in [-1, 1). */
static double splitmix_unit(unsigned long long i)
{
  unsigned long long z = (i + 1ULL) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

/* Plain BiCGStab (van der Vorst 1992) on A x = b where A already has unit
 * diagonal (rows scaled by their diagonal).  Stops when ||r|| <= rtol ||b||.
 * The shadow residual is a fixed pseudo-random vector: the textbook choice
 * r^ = r0 is supported only near the inlet for transport from a cold start,
 * and r^.r collapses as the residual moves downstream (breakdown). */
static int bicgstab(const stencil_t *A, const double *b, double *x, double rtol,
                    int maxit, int *its, double *relres, double *relres0)
{
  long N = A->N;
  double *r = malloc(N * sizeof(double)), *rh = malloc(N * sizeof(double));
  double *p = calloc(N, sizeof(double)), *v = calloc(N, sizeof(double));
  double *s = malloc(N * sizeof(double)), *t = malloc(N * sizeof(double));
  if (!r || !rh || !p || !v || !s || !t) {
    free(r); free(rh); free(p); free(v); free(s); free(t); return ORC_ERR_OOM;
  }
  double bnorm = sqrt(dot(N, b, b));
  stencil_apply(A, x, t);
  for (long i = 0; i < N; ++i) { r[i] = b[i] - t[i]; rh[i] = splitmix_unit((unsigned long long)i); }
  double rho = 1.0, alpha = 1.0, omega = 1.0;
  double rnorm = sqrt(dot(N, r, r));
  if (relres0) *relres0 = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  double tol = rtol * bnorm;
  int k = 0, status = ORC_ERR_NOCONV;
  while (1) {
    if (rnorm <= tol || rnorm == 0.0) { status = ORC_OK; break; }
    if (k >= maxit) break;
    double rho_new = dot(N, rh, r);
    if (rho_new == 0.0) break;
    double beta = (rho_new / rho) * (alpha / omega);
    rho = rho_new;
    for (long i = 0; i < N; ++i) p[i] = r[i] + beta * (p[i] - omega * v[i]);
    stencil_apply(A, p, v);
    double rv = dot(N, rh, v);
    if (rv == 0.0) break;
    alpha = rho / rv;
    for (long i = 0; i < N; ++i) s[i] = r[i] - alpha * v[i];
    double snorm = sqrt(dot(N, s, s));
    ++k;
    if (snorm <= tol) {
      for (long i = 0; i < N; ++i) x[i] += alpha * p[i];
      rnorm = snorm;
      continue;
    }
    stencil_apply(A, s, t);
    double tt = dot(N, t, t);
    if (tt == 0.0) break;
    omega = dot(N, t, s) / tt;
    for (long i = 0; i < N; ++i) { x[i] += alpha * p[i] + omega * s[i]; r[i] = s[i] - omega * t[i]; }
    rnorm = sqrt(dot(N, r, r));
    if (omega == 0.0) break;
  }
  *its = k;
  *relres = bnorm > 0.0 ? rnorm / bnorm : 0.0;
  free(r); free(rh); free(p); free(v); free(s); free(t);
  return status;
}

/* ---------------------------------------------------- S1: coefficients */

typedef struct {
  double *epsf[3];   /* face porosity */
  double *dmom[3];   /* eps_f-scaled momentum diagonal (1 on fixed faces) */
  double *af[3];     /* rho/(eps_f dt) + beta_f: pressure-correction coefficient (0 on fixed) */
  double *T[3];      /* pressure transmissibility S/(a_f d_f) (0 on fixed) */
  double *w[3];      /* reactive face velocity k_c n_f . S e_d (0 on boundaries) */
  double *g[3];      /* cell gradient of eps */
  double *gmag;      /* |grad eps| */
  double *nrm[3];    /* interface normal toward the solid, or 0 */
  double *psi;       /* localization function (psi models) */
  double lambda;
} coef_t;

static void coef_free(coef_t *C)
{
  for (int d = 0; d < 3; ++d) {
    free(C->epsf[d]); free(C->dmom[d]); free(C->af[d]); free(C->T[d]); free(C->w[d]);
    free(C->g[d]); free(C->nrm[d]);
  }
  free(C->gmag); free(C->psi);
  memset(C, 0, sizeof(*C));
}

static int coef_alloc(coef_t *C, const grid_t *g)
{
  memset(C, 0, sizeof(*C));
  for (int d = 0; d < 3; ++d) {
    C->epsf[d] = calloc(g->nf[d], sizeof(double));
    C->dmom[d] = calloc(g->nf[d], sizeof(double));
    C->af[d]   = calloc(g->nf[d], sizeof(double));
    C->T[d]    = calloc(g->nf[d], sizeof(double));
    C->w[d]    = calloc(g->nf[d], sizeof(double));
    C->g[d]    = calloc(g->nc, sizeof(double));
    C->nrm[d]  = calloc(g->nc, sizeof(double));
    if (!C->epsf[d] || !C->dmom[d] || !C->af[d] || !C->T[d] || !C->w[d] || !C->g[d] || !C->nrm[d])
      return ORC_ERR_OOM;
  }
  C->gmag = calloc(g->nc, sizeof(double));
  C->psi = calloc(g->nc, sizeof(double));
  if (!C->gmag || !C->psi) return ORC_ERR_OOM;
  return ORC_OK;
}

/* Kind of the Laplacian neighbour of the momentum unknown on face (d, x), in
 * direction e, side s.  Weights in the viscous diagonal: unknown 1, fixed
 * neighbour value 1, mirrored no-slip ghost 2, zero-gradient ghost 0. */
enum { NB_UNKNOWN, NB_FIXED, NB_GHOST, NB_ZEROGRAD };

static int mom_nb(const grid_t *g, int d, const int x[3], int e, int s,
                  double u_in, double *fixed_val)
{
  int y = x[e] + s;
  *fixed_val = 0.0;
  if (e == d) {
    if (d == 0) {
      if (y == 0 && !g->drive) { *fixed_val = u_in; return NB_FIXED; }   /* the inlet face */
      if (y > g->n[0] || y < 0) return NB_ZEROGRAD;             /* past the outlet / the inlet */
      return NB_UNKNOWN;
    }
    if (y == 0 || y == g->n[d]) return NB_FIXED;                /* wall face, u = 0 */
    return NB_UNKNOWN;
  }
  if (y >= 0 && y < g->n[e]) return NB_UNKNOWN;
  if (e == 0) return (y < 0) ? NB_GHOST : NB_ZEROGRAD;          /* inlet: no tangential velocity */
  return NB_GHOST;                                              /* no-slip wall */
}

static double nb_weight(int kind)
{
  switch (kind) {
    case NB_UNKNOWN: return 1.0;
    case NB_FIXED:   return 1.0;
    case NB_GHOST:   return 2.0;
    default:         return 0.0;
  }
}

static int compute_coefficients(const grid_t *g, const orc_prob *P, double dt,
                                const double *eps, coef_t *C)
{
  const double dx = g->dx, S = g->S;
  /* face quantities */
  for (int d = 0; d < g->nd; ++d) {
    for (long f = 0; f < g->nf[d]; ++f) {
      int x[3];
      unflatten(g->fd[d], f, x);
      int kind = face_kind(g, d, x[d]);
      int lo[3] = {x[0], x[1], x[2]}; lo[d] -= 1;
      double ef;
      if (kind == F_INTERIOR) ef = 0.5 * (eps[cidx(g, lo)] + eps[cidx(g, x)]);
      else if (x[d] == 0)     ef = eps[cidx(g, x)];
      else                    ef = eps[cidx(g, lo)];
      C->epsf[d][f] = ef;
      if (mom_unknown(g, d, x)) {
        double beta = P->mu * (1.0 - ef) * (1.0 - ef) / (P->k0 * ef * ef * ef);
        double nbsum = 0.0, fv;
        for (int e = 0; e < g->nd; ++e)
          for (int s = -1; s <= 1; s += 2) nbsum += nb_weight(mom_nb(g, d, x, e, s, P->u_in, &fv));
        double dm, af;
        if (P->simple) {
          /* steady momentum (Eq. momentumDBSQS) with implicit under-relaxation:
           * diagonal a / relax_u; the pressure correction of SIMPLE uses the
           * same (relaxed) diagonal, unscaled by eps_f */
          dm = (ef * beta + P->mu / (dx * dx) * nbsum) / P->relax_u;
          af = dm / ef;
        } else {
          dm = P->rho / dt + ef * beta + P->mu / (dx * dx) * nbsum;
          /* pressure-correction coefficient: the inertia + drag part of the
           * unscaled diagonal (incremental projection of the backward-Euler
           * step; the viscous part is left out so one pass per step is stable) */
          af = P->rho / (ef * dt) + beta;
        }
        double dist = (kind == F_OUTLET || kind == F_INLET) ? 0.5 * dx : dx;
        C->dmom[d][f] = dm;
        C->af[d][f] = af;
        C->T[d][f] = S / (af * dist);
      } else {
        C->dmom[d][f] = 1.0;
        C->af[d][f] = 0.0;
        C->T[d][f] = 0.0;
      }
    }
  }
  /* cell gradient of eps, zero-gradient at every boundary: central differences,
   * or (grad_scheme 1, a VoS-psi variant of Section 2.4) per direction the
   * one-sided difference toward the neighbour of larger eps, so that the area of
   * a sharp interface lands in the cell that holds the solid (ties: the + side).
   * The normal -grad/|grad| of Section 2.3 is taken as 0 where eps varies by
   * at most 1e-6 across a cell: eps is O(1) and stored to ~1e-16, so below that
   * the direction of the gradient is set by rounding, and a unit reactive flux
   * along it would turn rounding into acid sinks of order k_c c / dx */
  const double tau = 1e-6 / dx;
  for (long id = 0; id < g->nc; ++id) {
    int x[3];
    unflatten(g->n, id, x);
    double gg = 0.0;
    for (int d = 0; d < 3; ++d) C->g[d][id] = 0.0;
    for (int d = 0; d < g->nd; ++d) {
      int xm[3] = {x[0], x[1], x[2]}, xp[3] = {x[0], x[1], x[2]};
      xm[d] = x[d] > 0 ? x[d] - 1 : x[d];
      xp[d] = x[d] < g->n[d] - 1 ? x[d] + 1 : x[d];
      double gd;
      if (P->grad_scheme == 1) {
        double em = eps[cidx(g, xm)], ep = eps[cidx(g, xp)], e0 = eps[id];
        gd = (em > ep) ? (e0 - em) / dx : (ep - e0) / dx;
      } else {
        gd = (eps[cidx(g, xp)] - eps[cidx(g, xm)]) / (2.0 * dx);
      }
      C->g[d][id] = gd;
      gg += gd * gd;
    }
    double gm = sqrt(gg);
    C->gmag[id] = gm;
    for (int d = 0; d < 3; ++d) C->nrm[d][id] = (gm > tau) ? -C->g[d][id] / gm : 0.0;
  }
  /* reactive face velocity: mean of the two cell normals, zero on boundaries */
  for (int d = 0; d < g->nd; ++d) {
    for (long f = 0; f < g->nf[d]; ++f) {
      int x[3];
      unflatten(g->fd[d], f, x);
      if (face_kind(g, d, x[d]) != F_INTERIOR) { C->w[d][f] = 0.0; continue; }
      int lo[3] = {x[0], x[1], x[2]}; lo[d] -= 1;
      C->w[d][f] = P->kc * 0.5 * (C->nrm[d][cidx(g, lo)] + C->nrm[d][cidx(g, x)]) * S;
    }
  }
  /* localization function psi = lambda eps (1 - eps), or psi = 1 */
  double lam = 4.0;
  if (P->model == 2) {
    double num = 0.0, den = 0.0;
    for (long id = 0; id < g->nc; ++id) {
      num += C->gmag[id];
      den += C->gmag[id] * eps[id] * (1.0 - eps[id]);
    }
    lam = (den > 0.0) ? num / den : 4.0;
  }
  C->lambda = lam;
  for (long id = 0; id < g->nc; ++id)
    C->psi[id] = (P->psi_kind == 1) ? 1.0 : lam * eps[id] * (1.0 - eps[id]);
  return ORC_OK;
}

/* ----------------------------------------------------- S2: momentum */

/* u_d / eps_f on face (d, y) of the d face grid. */
static double conv_phi(const grid_t *g, const coef_t *C, double *const u[3], int d, const int y[3])
{
  long f = fidx(g, d, y);
  return u[d][f] / C->epsf[d][f];
}

/* Momentum convection of Eq. momentumDBS, explicit first-order upwind, on the
 * interior face (d, x): rho [div(u u / eps)]_f, i.e. the eps_f-scaled row's
 * convection term.  The control volume is the cell-sized box centred on the
 * face.  Across its two faces normal to d (at the centres of the cells on
 * either side) the transport velocity is the mean of that cell's two d-faces;
 * across its faces normal to e != d it is the mean of the two e-faces of the
 * cells on either side of face (d, x) in that plane.  The transported value
 * u_d / eps_f is the control volume's own when the flux leaves it, else the
 * neighbouring d-face's; beyond the domain the inflowing value is 0 (walls and
 * the inlet carry no tangential momentum) and at the outlet plane the own value
 * (zero gradient). */
static double conv_face(const grid_t *g, const orc_prob *P, const coef_t *C, double *const u[3],
                        int d, const int x[3])
{
  double flux = 0.0;
  const double own = conv_phi(g, C, u, d, x);
  for (int e = 0; e < g->nd; ++e)
    for (int s = -1; s <= 1; s += 2) {
      int xn[3] = {x[0], x[1], x[2]};
      xn[e] += s;
      double U, nb;
      if (e == d) {
        /* the neighbouring d-face exists: x is interior in d */
        U = 0.5 * (u[d][fidx(g, d, x)] + u[d][fidx(g, d, xn)]);
        nb = conv_phi(g, C, u, d, xn);
      } else {
        int q = x[e] + (s > 0);                 /* plane of e-faces */
        int cl[3] = {x[0], x[1], x[2]}, cu[3] = {x[0], x[1], x[2]};
        cl[d] -= 1;
        cl[e] = q; cu[e] = q;
        U = 0.5 * (u[e][fidx(g, e, cl)] + u[e][fidx(g, e, cu)]);
        if (xn[e] >= 0 && xn[e] < g->n[e]) nb = conv_phi(g, C, u, d, xn);
        else nb = (e == 0 && s > 0) ? own : 0.0;
      }
      double out = s * U;
      flux += out * (out >= 0.0 ? own : nb);
    }
  return P->rho * flux / g->dx;
}

/* Assemble the eps_f-scaled momentum system of component d on its face grid.
 * Fixed faces (inlet, walls) are identity rows with zero right-hand side.
 * un: the velocity the inertia (one pass) or relaxation (SIMPLE) term and the
 * convection are taken from; pn: the pressure whose gradient drives it. */
static void assemble_momentum(const grid_t *g, const orc_prob *P, double dt, const coef_t *C,
                              int d, double *const un[3], const double *pn, stencil_t *A, double *b)
{
  const double dx = g->dx, cvis = P->mu / (dx * dx);
  for (long f = 0; f < g->nf[d]; ++f) {
    int x[3];
    unflatten(g->fd[d], f, x);
    for (int k = 0; k < 7; ++k) A->a[k][f] = 0.0;
    if (!mom_unknown(g, d, x)) { A->a[0][f] = 1.0; b[f] = 0.0; continue; }
    A->a[0][f] = C->dmom[d][f];
    /* inertia rho/dt u^n (one pass), or the relaxation term (1 - r)/r a u^k (SIMPLE) */
    double rhs = P->simple ? C->dmom[d][f] * (1.0 - P->relax_u) * un[d][f] : P->rho / dt * un[d][f];
    for (int e = 0; e < g->nd; ++e)
      for (int s = -1; s <= 1; s += 2) {
        double fv;
        int kind = mom_nb(g, d, x, e, s, P->u_in, &fv);
        if (kind == NB_UNKNOWN) A->a[1 + 2 * e + (s > 0)][f] = -cvis;
        else if (kind == NB_FIXED) rhs += cvis * fv;
      }
    /* old pressure gradient across the face */
    int kind = face_kind(g, d, x[d]);
    double pl, pu, dist;
    if (kind == F_OUTLET) {
      int lo[3] = {x[0], x[1], x[2]}; lo[d] -= 1;
      pl = pn[cidx(g, lo)]; pu = P->p_out; dist = 0.5 * dx;
    } else if (kind == F_INLET) {
      pl = P->p_in; pu = pn[cidx(g, x)]; dist = 0.5 * dx;
    } else {
      int lo[3] = {x[0], x[1], x[2]}; lo[d] -= 1;
      pl = pn[cidx(g, lo)]; pu = pn[cidx(g, x)]; dist = dx;
    }
    rhs -= C->epsf[d][f] * (pu - pl) / dist;
    if (P->convection && kind == F_INTERIOR) rhs -= conv_face(g, P, C, un, d, x);
    b[f] = rhs;
  }
}

/* ------------------------------------------------------ S3: pressure */

static void assemble_pressure_matrix(const grid_t *g, const coef_t *C, stencil_t *A)
{
  for (long id = 0; id < g->nc; ++id) {
    int x[3];
    unflatten(g->n, id, x);
    for (int k = 0; k < 7; ++k) A->a[k][id] = 0.0;
    for (int d = 0; d < g->nd; ++d)
      for (int s = -1; s <= 1; s += 2) {
        int xf[3] = {x[0], x[1], x[2]};
        xf[d] += (s > 0);
        int kind = face_kind(g, d, xf[d]);
        double T = C->T[d][fidx(g, d, xf)];
        if (kind == F_INTERIOR) { A->a[0][id] += T; A->a[1 + 2 * d + (s > 0)][id] = -T; }
        else if (kind == F_OUTLET || (kind == F_INLET && g->drive)) A->a[0][id] += T;
      }
  }
}

/* Outward volume flux sum S u . n over the faces of every cell. */
static void divergence(const grid_t *g, double *const u[3], double *div)
{
  for (long id = 0; id < g->nc; ++id) {
    int x[3];
    unflatten(g->n, id, x);
    double s = 0.0;
    for (int d = 0; d < g->nd; ++d) {
      int xu[3] = {x[0], x[1], x[2]};
      xu[d] += 1;
      s += u[d][fidx(g, d, xu)] - u[d][fidx(g, d, x)];
    }
    div[id] = s * g->S;
  }
}

/* --------------------------------------------------------- S5: transport */

/* van Leer (1974) correction to the upwind face value of phi on interior face
 * (d, x), for a face velocity of sign vel.  With C the upwind cell, D the
 * downwind cell and U the cell upwind of C:  a = phi_C - phi_U,
 * b = phi_D - phi_C, face value = phi_C + (a b > 0 ? a b / (a + b) : 0).
 * A missing U (boundary) takes the zero-gradient ghost phi_U = phi_C. */
static double vl_corr(const grid_t *g, const double *phi, int d, const int x[3], double vel)
{
  int lo[3] = {x[0], x[1], x[2]}; lo[d] -= 1;
  int cu[3] = {x[0], x[1], x[2]}, cc[3], cd[3];
  if (vel >= 0.0) {
    memcpy(cc, lo, sizeof cc); memcpy(cd, x, sizeof cd);
    cu[d] = x[d] - 2;
  } else {
    memcpy(cc, x, sizeof cc); memcpy(cd, lo, sizeof cd);
    cu[d] = x[d] + 1;
  }
  double pc = phi[cidx(g, cc)], pd = phi[cidx(g, cd)];
  double pu = (cu[d] < 0 || cu[d] >= g->n[d]) ? pc : phi[cidx(g, cu)];
  double a = pc - pu, b = pd - pc;
  return (a * b > 0.0) ? a * b / (a + b) : 0.0;
}

static double upwind_value(const grid_t *g, const double *phi, int d, const int x[3], double vel)
{
  int lo[3] = {x[0], x[1], x[2]}; lo[d] -= 1;
  return vel >= 0.0 ? phi[cidx(g, lo)] : phi[cidx(g, x)];
}

/* Transport system (not yet row-scaled).  u: corrected face velocities;
 * cold: the field the deferred corrections lag on (c^n, or in the SIMPLE loop
 * the previous outer iterate).  Transient storage (P->transient):
 * (eps c - eps_prev c0) V / dt with eps the step's porosity, eps_prev the
 * previous step's and c0 the concentration at the step's start (may be NULL
 * otherwise).  SIMPLE under-relaxation relax_c < 1: diagonal / relax_c and
 * (1 - relax_c)/relax_c diagonal * cold on the right-hand side. */
static void assemble_transport(const grid_t *g, const orc_prob *P, const coef_t *C,
                               const double *eps, double *const u[3], const double *cold,
                               const double *eps_prev, const double *c0, double dt,
                               stencil_t *A, double *b)
{
  const double S = g->S, dx = g->dx, V = g->V;
  for (long id = 0; id < g->nc; ++id) {
    int x[3];
    unflatten(g->n, id, x);
    for (int k = 0; k < 7; ++k) A->a[k][id] = 0.0;
    double rhs = 0.0;
    for (int d = 0; d < g->nd; ++d)
      for (int s = -1; s <= 1; s += 2) {
        int xf[3] = {x[0], x[1], x[2]};
        xf[d] += (s > 0);
        long f = fidx(g, d, xf);
        int kind = face_kind(g, d, xf[d]);
        int slot = 1 + 2 * d + (s > 0);
        double Fo = s * S * u[d][f];                   /* outward volume flux */
        if (kind == F_INTERIOR) {
          /* convection: implicit upwind + lagged van Leer correction */
          if (Fo >= 0.0) A->a[0][id] += Fo; else A->a[slot][id] += Fo;
          rhs -= Fo * vl_corr(g, cold, d, xf, u[d][f]);
          /* diffusion, eps_f D S / dx */
          double G = P->D * C->epsf[d][f] * S / dx;
          A->a[0][id] += G; A->a[slot][id] -= G;
          /* iVoS acid sink: eps_P * outward reactive flux of c (upwind along w + lagged correction) */
          if (P->model == 0) {
            double wo = s * C->w[d][f];
            double k = P->zeta * eps[id] * wo;
            if (wo >= 0.0) A->a[0][id] += k; else A->a[slot][id] += k;
            rhs -= k * vl_corr(g, cold, d, xf, C->w[d][f]);
          }
        } else if (kind == F_INLET) {
          /* convective inflow of c_in (an outflow through the inlet leaves with c_P) */
          if (Fo < 0.0) rhs -= Fo * P->c_in; else A->a[0][id] += Fo;
          double G = P->D * eps[id] * S / (0.5 * dx);    /* Dirichlet at the face */
          A->a[0][id] += G; rhs += G * P->c_in;
        } else if (kind == F_OUTLET) {
          A->a[0][id] += Fo;                             /* zero gradient: c_f = c_P */
        }
      }
    if (P->model != 0) A->a[0][id] += P->zeta * P->kc * C->psi[id] * C->gmag[id] * V;
    if (P->transient) {
      A->a[0][id] += eps[id] * V / dt;
      rhs += eps_prev[id] * c0[id] * V / dt;
    }
    if (P->simple && P->relax_c < 1.0) {
      double dg = A->a[0][id] / P->relax_c;
      rhs += (dg - A->a[0][id]) * cold[id];
      A->a[0][id] = dg;
    }
    b[id] = rhs;
  }
}

/* ------------------------------------------------------ S6: reaction rate */

/* Rbar per cell (mol/m3/s) and the acid sink per cell (mol/s, before zeta).
 * iVoS (Eq. RfiVoS): Rbar V = eps_P sum_f w_f c^R_f - sum_f w_f (eps c)^R_f, with
 * c^R_f the face values the transport solve used (upwind of c^{n+1} plus the
 * van Leer correction lagged on c^n) and (eps c)^R_f the van Leer face value of
 * eps^n c^{n+1}; the acid sink is the first term (fluid side).
 * VoS-psi / psi' (Eq. RfVoSpsi): Rbar = k_c c psi |grad eps|, sink = Rbar V. */
static void reaction_rates(const grid_t *g, const orc_prob *P, const coef_t *C,
                           const double *eps, const double *c_new, const double *c_old,
                           double *rbar, double *sink)
{
  double *q = malloc(g->nc * sizeof(double));
  for (long i = 0; i < g->nc; ++i) q[i] = eps[i] * c_new[i];
  for (long id = 0; id < g->nc; ++id) {
    int x[3];
    unflatten(g->n, id, x);
    double R, sk;
    if (P->model == 0) {
      double t1 = 0.0, t2 = 0.0;
      for (int d = 0; d < g->nd; ++d)
        for (int s = -1; s <= 1; s += 2) {
          int xf[3] = {x[0], x[1], x[2]};
          xf[d] += (s > 0);
          if (face_kind(g, d, xf[d]) != F_INTERIOR) continue;
          long f = fidx(g, d, xf);
          double wf = C->w[d][f], wo = s * wf;
          t1 += wo * (upwind_value(g, c_new, d, xf, wf) + vl_corr(g, c_old, d, xf, wf));
          t2 += wo * (upwind_value(g, q, d, xf, wf) + vl_corr(g, q, d, xf, wf));
        }
      sk = eps[id] * t1;
      R = sk - t2;
    } else {
      sk = P->kc * C->psi[id] * C->gmag[id] * c_new[id] * g->V;
      R = sk;
    }
    rbar[id] = R / g->V;
    sink[id] = sk;
  }
  free(q);
}

/* ------------------------------------------------------------- the step */

static void get_face_arrays(double *ux, double *uy, double *uz, double *u[3])
{
  u[0] = ux; u[1] = uy; u[2] = uz;
}

int orc_eps_from_solid(const orc_prob *P, const double *eps_s, double *eps)
{
  long n = (long)P->nx * P->ny * P->nz;
  for (long i = 0; i < n; ++i) {
    double e = 1.0 - eps_s[i];
    if (e < P->eps_min) e = P->eps_min;
    if (e > 1.0) e = 1.0;
    eps[i] = e;
  }
  return ORC_OK;
}

static int check_prob(const orc_prob *P, double dt)
{
  if (P->nx < 2 || P->ny < 1 || P->nz < 1 || P->dx <= 0.0 || dt <= 0.0) return ORC_ERR_ARG;
  if (P->mu <= 0.0 || P->rho <= 0.0 || P->k0 <= 0.0 || P->eps_min <= 0.0) return ORC_ERR_ARG;
  if (!(P->deps_max >= 0.0)) return ORC_ERR_ARG;
  if (P->model < 0 || P->model > 2) return ORC_ERR_ARG;
  if (P->drive != 0 && P->drive != 1) return ORC_ERR_ARG;
  if (P->grad_scheme != 0 && P->grad_scheme != 1) return ORC_ERR_ARG;
  if (P->grad_scheme == 1 && P->model == 0) return ORC_ERR_ARG;  /* decentred: VoS-psi variants only */
  if (P->psi_kind != 0 && P->psi_kind != 1) return ORC_ERR_ARG;
  if (P->psi_kind == 1 && P->model == 2) return ORC_ERR_ARG;     /* lambda is fitted to eps (1 - eps) */
  if (!(P->solid_dt >= 0.0) || P->solid_dt > 1e300) return ORC_ERR_ARG;
  if (P->solid_dt > 0.0 && P->transient) return ORC_ERR_ARG;   /* the storage terms take dt */
  if (P->simple) {
    if (P->outer_max < 1 || !(P->outer_tol >= 0.0)) return ORC_ERR_ARG;
    if (!(P->relax_u > 0.0 && P->relax_u <= 1.0) || !(P->relax_p > 0.0 && P->relax_p <= 1.0) ||
        !(P->relax_c > 0.0 && P->relax_c <= 1.0)) return ORC_ERR_ARG;
  }
  return ORC_OK;
}

/* Time step of the solid update (Appendix D): the nominal step T -- dt, or
 * solid_dt when that is set (Appendix A's quasi-static reading: flow and
 * transport are steady, so dt is then only the flow's pseudo time step and the
 * solid interface alone sets the physical step) -- or with deps_max > 0
 * min(T, deps_max / max |Vm Rbar|) where the maximum runs over the cells whose
 * distance to the clip bound in the direction of their change exceeds deps_max
 * (a cell closer to its bound changes by at most that distance anyway). */
static double solid_dt(const grid_t *g, const orc_prob *P, double dt, const double *eps, const double *rbar)
{
  if (P->solid_dt > 0.0) dt = P->solid_dt;
  double dts = dt;
  if (P->deps_max > 0.0) {
    double m = 0.0;
    for (long id = 0; id < g->nc; ++id) {
      double r = P->Vm * rbar[id];
      double room = r > 0.0 ? 1.0 - eps[id] : eps[id] - P->eps_min;
      double a = fabs(r);
      if (room > P->deps_max && a > m) m = a;
    }
    if (m > 0.0) {
      double lim = P->deps_max / m;
      dts = lim < dt ? lim : dt;
    }
  }
  return dts;
}

/* Momentum predictor of every component from the state (u, p) (S2). */
static int momentum_stage(const grid_t *g, const orc_prob *P, double dt, const coef_t *C,
                          double *const u[3], const double *p, double *const ustar[3],
                          orc_diag *dd, double *r0max)
{
  int status = ORC_OK;
  for (int d = 0; d < g->nd; ++d) {
    stencil_t A;
    double *b = calloc(g->nf[d], sizeof(double));
    if (stencil_alloc(&A, g->fd[d]) || !b) { stencil_free(&A); free(b); return ORC_ERR_OOM; }
    assemble_momentum(g, P, dt, C, d, u, p, &A, b);
    for (long f = 0; f < g->nf[d]; ++f) {
      int x[3];
      unflatten(g->fd[d], f, x);
      ustar[d][f] = mom_unknown(g, d, x) ? u[d][f] : 0.0;
    }
    double r0 = 0.0;
    int s2 = pcg_jacobi(&A, b, ustar[d], P->rtol_u, P->maxit_u, &dd->it_u[d], &dd->res_u[d], &r0);
    if (s2 && !status) status = s2;
    if (r0 > *r0max) *r0max = r0;
    /* restore the fixed faces */
    for (long f = 0; f < g->nf[d]; ++f) {
      int x[3];
      unflatten(g->fd[d], f, x);
      if (!mom_unknown(g, d, x)) ustar[d][f] = (d == 0 && x[0] == 0) ? P->u_in : 0.0;
    }
    stencil_free(&A); free(b);
  }
  return status;
}

/* One full step S1..S7.  eps, ux, uy, uz, p, c are updated in place (aux too
 * when given).  One pass of S2..S6, or with P->simple the SIMPLE loop of
 * Appendix B over them with eps frozen, until every solve starts within
 * outer_tol of its solution. */
int orc_step(const orc_prob *P, double dt, double *eps, double *ux, double *uy, double *uz,
             double *p, double *c, orc_aux *aux, orc_out *out, orc_diag *dg)
{
  int st = check_prob(P, dt);
  if (st) return st;
  if (P->transient && (!aux || !aux->eps_prev || !aux->rbar_prev)) return ORC_ERR_ARG;
  grid_t g;
  grid_init(&g, P);
  double *u[3];
  get_face_arrays(ux, uy, uz, u);
  orc_diag dd;
  memset(&dd, 0, sizeof dd);
  const double S = g.S, V = g.V;

  coef_t C;
  if ((st = coef_alloc(&C, &g))) { coef_free(&C); return st; }
  compute_coefficients(&g, P, dt, eps, &C);
  dd.lambda = C.lambda;

  int status = ORC_OK;
  double *ustar[3] = {NULL, NULL, NULL};
  double *pn = malloc(g.nc * sizeof(double)), *rhs = malloc(g.nc * sizeof(double));
  double *div = malloc(g.nc * sizeof(double)), *c0 = malloc(g.nc * sizeof(double));
  double *cold = malloc(g.nc * sizeof(double)), *rsrc = calloc(g.nc, sizeof(double));
  double *bsc = malloc(g.nc * sizeof(double));
  double *rbar = out && out->rbar ? out->rbar : malloc(g.nc * sizeof(double));
  double *sink = out && out->sink ? out->sink : malloc(g.nc * sizeof(double));
  stencil_t Ap, At, As;
  memset(&Ap, 0, sizeof Ap); memset(&At, 0, sizeof At); memset(&As, 0, sizeof As);
  for (int d = 0; d < 3; ++d) {
    ustar[d] = calloc(g.nf[d], sizeof(double));
    if (!ustar[d]) status = ORC_ERR_OOM;
  }
  if (status || !pn || !rhs || !div || !c0 || !cold || !rsrc || !bsc || !rbar || !sink ||
      stencil_alloc(&Ap, g.n) || stencil_alloc(&At, g.n) || stencil_alloc(&As, g.n)) {
    status = ORC_ERR_OOM;
    goto done;
  }
  memcpy(c0, c, g.nc * sizeof(double));
  if (P->transient) memcpy(rsrc, aux->rbar_prev, g.nc * sizeof(double));
  const double *eps_prev = P->transient ? aux->eps_prev : NULL;
  /* continuity source coefficient of Eq. contDBS: div u = Rbar M_ws (1/rho_s - 1/rho) */
  const double srcc = P->Vm - P->Vm_f;
  assemble_pressure_matrix(&g, &C, &Ap);

  const int nout = P->simple ? P->outer_max : 1;
  for (int it = 0; it < nout; ++it) {
    double r0max = 0.0, r0 = 0.0;
    /* S2: momentum predictor per component, started from the current u */
    int s2 = momentum_stage(&g, P, dt, &C, u, p, ustar, &dd, &r0max);
    if (s2 == ORC_ERR_OOM) { status = s2; goto done; }
    if (s2 && !status) status = s2;

    /* S3: pressure, A p = -div(u*) + A p^k (+ source V), started from p^k */
    memcpy(pn, p, g.nc * sizeof(double));
    divergence(&g, ustar, div);
    stencil_apply(&Ap, pn, rhs);
    for (long i = 0; i < g.nc; ++i) rhs[i] -= div[i];
    if (P->transient)
      for (long i = 0; i < g.nc; ++i) rhs[i] += srcc * rsrc[i] * V;
    int s3 = pcg_jacobi(&Ap, rhs, p, P->rtol_p, P->maxit_p, &dd.it_p, &dd.res_p, &r0);
    if (s3 && !status) status = s3;
    if (r0 > r0max) r0max = r0;

    /* S4: velocity correction on the momentum unknowns; fixed faces keep their values */
    for (int d = 0; d < g.nd; ++d) {
      for (long f = 0; f < g.nf[d]; ++f) {
        int x[3];
        unflatten(g.fd[d], f, x);
        if (!mom_unknown(&g, d, x)) { u[d][f] = ustar[d][f]; continue; }
        int kind = face_kind(&g, d, x[d]);
        double dpl, dpu, dist;
        if (kind == F_INLET) {
          long U = cidx(&g, x);
          dpl = 0.0; dpu = p[U] - pn[U]; dist = 0.5 * g.dx;
        } else {
          int lo[3] = {x[0], x[1], x[2]}; lo[d] -= 1;
          long L = cidx(&g, lo);
          dpl = p[L] - pn[L];
          if (kind == F_OUTLET) { dpu = 0.0; dist = 0.5 * g.dx; }
          else { long U = cidx(&g, x); dpu = p[U] - pn[U]; dist = g.dx; }
        }
        u[d][f] = ustar[d][f] - (dpu - dpl) / (C.af[d][f] * dist);
      }
    }
    /* SIMPLE: explicit under-relaxation of the pressure (the velocity keeps the full correction) */
    if (P->simple)
      for (long i = 0; i < g.nc; ++i) p[i] = pn[i] + P->relax_p * (p[i] - pn[i]);

    /* S5: quasi-static (or transient) transport, row-scaled BiCGStab, started from c^k */
    memcpy(cold, c, g.nc * sizeof(double));
    assemble_transport(&g, P, &C, eps, u, cold, eps_prev, c0, dt, &At, rhs);
    for (long i = 0; i < g.nc; ++i) {
      double dgl = At.a[0][i];
      for (int k = 0; k < 7; ++k) As.a[k][i] = At.a[k][i] / dgl;
      bsc[i] = rhs[i] / dgl;
    }
    int s5 = bicgstab(&As, bsc, c, P->rtol_c, P->maxit_c, &dd.it_c, &dd.res_c, &r0);
    if (s5 && !status) status = s5;
    if (r0 > r0max) r0max = r0;

    /* S6: reaction rate from this iterate (recomputed every outer iteration, Appendix B) */
    reaction_rates(&g, P, &C, eps, c, cold, rbar, sink);
    dd.outer_its = it + 1;
    dd.outer_res = r0max;
    if (P->transient) {
      double sv = 0.0;
      for (long i = 0; i < g.nc; ++i) sv += srcc * rsrc[i] * V;
      dd.div_source = sv;
      memcpy(rsrc, rbar, g.nc * sizeof(double));   /* the next outer iteration's source */
    }
    if (P->simple && r0max <= P->outer_tol) break;
  }

  /* S7: solid update and diagnostics */
  {
    double acid_sink = 0.0, solid_rate = 0.0;
    for (long id = 0; id < g.nc; ++id) { acid_sink += sink[id]; solid_rate += rbar[id] * V; }
    /* boundary fluxes and pore averages use eps^n, as the transport solve did */
    double ain = 0.0, aout = 0.0, pin = 0.0, cg = 0.0, ec = 0.0, area = 0.0, qin = 0.0, acc = 0.0;
    int nin = 0;
    for (long id = 0; id < g.nc; ++id) {
      int x[3];
      unflatten(g.n, id, x);
      if (x[0] == 0) {
        int xf[3] = {0, x[1], x[2]};
        double ui = u[0][fidx(&g, 0, xf)];
        ain += S * ui * (ui > 0.0 ? P->c_in : c[id]) + P->D * eps[id] * S / (0.5 * g.dx) * (P->c_in - c[id]);
        qin += S * ui;
        pin += p[id];
        ++nin;
      }
      if (x[0] == g.n[0] - 1) {
        int xf[3] = {g.n[0], x[1], x[2]};
        aout += S * u[0][fidx(&g, 0, xf)] * c[id];
      }
      cg += c[id] * C.gmag[id] * V;
      ec += eps[id] * c[id] * V;
      area += C.gmag[id] * V;
      if (P->transient) acc += (eps[id] * c[id] - eps_prev[id] * c0[id]) * V / dt;
    }
    /* Appendix D: the largest change of the fluid fraction in a step is held
       to deps_max, here by shortening the solid update's step when the rates
       just computed would exceed it: dt_s = min(dt, deps_max / max |Vm Rbar|),
       the maximum over the cells the clip does not hold within deps_max of
       their bound (any other cell changes by at most its distance to the
       bound, itself <= deps_max) */
    double dts = solid_dt(&g, P, dt, eps, rbar);
    if (P->transient) memcpy(aux->eps_prev, eps, g.nc * sizeof(double));
    double clipped = 0.0, maxd = 0.0, dvol = 0.0, sv = 0.0, por = 0.0;
    for (long id = 0; id < g.nc; ++id) {
      double e0 = eps[id];
      double e1 = e0 + dts * P->Vm * rbar[id];
      double ec1 = e1 < P->eps_min ? P->eps_min : (e1 > 1.0 ? 1.0 : e1);
      clipped += (e1 - ec1) * V;
      dvol += (ec1 - e0) * V;
      double ad = fabs(ec1 - e0);
      if (ad > maxd) maxd = ad;
      eps[id] = ec1;
      sv += (1.0 - ec1) * V;
      por += ec1;
    }
    if (P->transient) memcpy(aux->rbar_prev, rbar, g.nc * sizeof(double));
    dd.solid_volume = sv;
    dd.surface_area = area;
    dd.porosity = por / (double)g.nc;
    dd.U_D = qin / ((double)g.n[1] * g.n[2] * S);
    if (P->drive) {
      dd.dP = P->p_in - P->p_out;
      dd.K = dd.dP != 0.0 ? P->mu * dd.U_D * g.n[0] * g.dx / dd.dP : 0.0;
    } else {
      dd.dP = pin / nin - P->p_out;
      dd.K = dd.dP != 0.0 ? P->mu * P->u_in * (g.n[0] - 0.5) * g.dx / dd.dP : 0.0;
    }
    dd.acid_in = ain;
    dd.acid_out = aout;
    dd.acid_consumed = P->zeta * acid_sink;
    dd.acid_accum = acc;
    dd.solid_rate = solid_rate;
    dd.acid_balance_rel = ain != 0.0 ? (ain - aout - dd.acid_consumed - acc) / ain : 0.0;
    double ref = dts * P->Vm * fabs(solid_rate);
    dd.solid_balance_rel = ref > 0.0 ? (dvol - dts * P->Vm * solid_rate + clipped) / ref : 0.0;
    dd.dt_solid = dts;
    dd.clipped_volume = clipped;
    dd.max_deps = maxd;
    dd.R_omega = (P->Vm > 0.0) ? dvol / ((double)g.nc * V) / (P->Vm * dts) : 0.0;
    double a = area / (g.nc * V);
    dd.alpha = (a > 0.0 && ec > 0.0) ? cg / (a * ec) : 0.0;
  }
  if (out) {
    for (int d = 0; d < 3; ++d)
      if (out->ustar[d]) memcpy(out->ustar[d], ustar[d], g.nf[d] * sizeof(double));
    if (out->gmag) memcpy(out->gmag, C.gmag, g.nc * sizeof(double));
  }
done:
  if (!(out && out->rbar)) free(rbar);
  if (!(out && out->sink)) free(sink);
  free(pn); free(rhs); free(div); free(c0); free(cold); free(rsrc); free(bsc);
  stencil_free(&Ap); stencil_free(&At); stencil_free(&As);
  for (int d = 0; d < 3; ++d) free(ustar[d]);
  coef_free(&C);
  if (dg) *dg = dd;
  return status;
}

/* ----------------------------------------- entry points used by the pins */

/* Assemble one of the step's linear systems from a given state, as dense-able
 * 7-point stencils.  which: 0,1,2 momentum component (u = u^n, p = p^n);
 * 3 pressure (u = u*, p = p^n); 4 transport (u = corrected velocities,
 * c = c^n, unscaled rows).  aux (may be NULL) supplies eps_prev for the
 * storage term (else eps) and rbar_prev for the continuity source (else 0).
 * stencil_out holds 7 arrays of n entries laid end to end (n = faces of that
 * component or cells), rhs_out n entries. */
int orc_assemble(const orc_prob *P, double dt, const double *eps, double *ux, double *uy,
                 double *uz, const double *p, const double *c, const orc_aux *aux, int which,
                 double *stencil_out, double *rhs_out)
{
  int st = check_prob(P, dt);
  if (st) return st;
  grid_t g;
  grid_init(&g, P);
  if (which < 0 || which > 4 || (which == 2 && g.nd == 2)) return ORC_ERR_ARG;
  double *u[3];
  get_face_arrays(ux, uy, uz, u);
  coef_t C;
  if ((st = coef_alloc(&C, &g))) { coef_free(&C); return st; }
  compute_coefficients(&g, P, dt, eps, &C);
  stencil_t A;
  const int *dims = which < 3 ? g.fd[which] : g.n;
  if (stencil_alloc(&A, dims)) { stencil_free(&A); coef_free(&C); return ORC_ERR_OOM; }
  long N = A.N;
  if (which < 3) {
    assemble_momentum(&g, P, dt, &C, which, u, p, &A, rhs_out);
  } else if (which == 3) {
    assemble_pressure_matrix(&g, &C, &A);
    double *div = malloc(N * sizeof(double));
    divergence(&g, u, div);
    stencil_apply(&A, p, rhs_out);
    for (long i = 0; i < N; ++i) rhs_out[i] -= div[i];
    if (P->transient && aux && aux->rbar_prev)
      for (long i = 0; i < N; ++i) rhs_out[i] += (P->Vm - P->Vm_f) * aux->rbar_prev[i] * g.V;
    free(div);
  } else {
    const double *ep = (aux && aux->eps_prev) ? aux->eps_prev : eps;
    assemble_transport(&g, P, &C, eps, u, c, ep, c, dt, &A, rhs_out);
  }
  for (int k = 0; k < 7; ++k) memcpy(stencil_out + k * N, A.a[k], N * sizeof(double));
  stencil_free(&A);
  coef_free(&C);
  return ORC_OK;
}

/* The oracle's own Krylov solvers on an arbitrary stencil (kind 0: Jacobi-PCG,
 * 1: BiCGStab on rows scaled here by their diagonal). */
int orc_solve_stencil(const int n[3], const double *stencil, const double *b, double *x,
                      int kind, double rtol, int maxit, int *its, double *relres)
{
  stencil_t A;
  if (stencil_alloc(&A, n)) { stencil_free(&A); return ORC_ERR_OOM; }
  long N = A.N;
  for (int k = 0; k < 7; ++k) memcpy(A.a[k], stencil + k * N, N * sizeof(double));
  int st;
  if (kind == 0) {
    st = pcg_jacobi(&A, b, x, rtol, maxit, its, relres, NULL);
  } else {
    double *bs = malloc(N * sizeof(double));
    for (long i = 0; i < N; ++i) {
      double dg = A.a[0][i];
      for (int k = 0; k < 7; ++k) A.a[k][i] /= dg;
      bs[i] = b[i] / dg;
    }
    st = bicgstab(&A, bs, x, rtol, maxit, its, relres, NULL);
    free(bs);
  }
  stencil_free(&A);
  return st;
}

/* S1 + S6 + the solid update alone with a prescribed concentration field
 * (frozen-c pins): c_new is the transported field, c_old the field the
 * corrections lag on.  Writes Rbar (per cell), the updated, clipped eps (in
 * place; its step shortened by deps_max as in a full step) and that step. */
int orc_reaction(const orc_prob *P, double dt, double *eps, const double *c_new,
                 const double *c_old, double *rbar, double *sink, double *gmag,
                 double *lambda_out, double *dts_out)
{
  int st = check_prob(P, dt);
  if (st) return st;
  grid_t g;
  grid_init(&g, P);
  coef_t C;
  if ((st = coef_alloc(&C, &g))) { coef_free(&C); return st; }
  compute_coefficients(&g, P, dt, eps, &C);
  double *sk = sink ? sink : malloc(g.nc * sizeof(double));
  reaction_rates(&g, P, &C, eps, c_new, c_old, rbar, sk);
  if (!sink) free(sk);
  double dts = solid_dt(&g, P, dt, eps, rbar);
  for (long id = 0; id < g.nc; ++id) {
    double e1 = eps[id] + dts * P->Vm * rbar[id];
    eps[id] = e1 < P->eps_min ? P->eps_min : (e1 > 1.0 ? 1.0 : e1);
  }
  if (gmag) memcpy(gmag, C.gmag, g.nc * sizeof(double));
  if (lambda_out) *lambda_out = C.lambda;
  if (dts_out) *dts_out = dts;
  coef_free(&C);
  return ORC_OK;
}

/* van Leer face value phi_C + a b / (a + b) exposed for the limiter pins. */
double orc_vanleer_face(double phi_u, double phi_c, double phi_d)
{
  double a = phi_c - phi_u, b = phi_d - phi_c;
  return phi_c + ((a * b > 0.0) ? a * b / (a + b) : 0.0);
}

/* Macroscopic reaction rate of Section 3.3: R_Omega = rho_s dphi / (M_w dt). */
double orc_r_omega(double rho_s, double M_w, double dphi, double dt)
{
  return rho_s * dphi / (M_w * dt);
}
