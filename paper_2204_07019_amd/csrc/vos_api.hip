// vos_api.hip -- host orchestration of the gfx950 Volume-of-Solid step and
// the C ABI declared in include/vos.h.
//
// Everything runs on the caller's stream.  Krylov scalars (alpha, beta, rho,
// omega, residuals, the convergence flag) live in device memory and are
// produced by one-block kernels, so a solve is a fixed sequence of launches
// per iteration with no host round trip; the host reads the flag every
// `check_every` iterations.  Once the flag is set every remaining kernel of
// the solve returns immediately, so over-launched iterations change nothing.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <type_traits>

#include "vos.h"
#include "vos_device.h"
#include "vos_internal.h"
#include "vos_kernels.h"
#include "vos_mg.h"
#include "vos_smg.h"
#include "vos_vcycle.h"
#include "vos_march3d.h"

using namespace vos;

namespace {

thread_local std::string g_err;

vos_status fail(vos_status st, const std::string &msg)
{
  g_err = msg;
  return st;
}

#define HIP_TRY(expr)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(VOS_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

constexpr size_t ALIGN = 256;

struct Plan {
  size_t off = 0;
  size_t take(size_t bytes)
  {
    size_t o = off;
    off += (bytes + ALIGN - 1) / ALIGN * ALIGN;
    return o;
  }
};

// Tile height of the tiled 2-D V-cycle kernels on a level of nc cells.
// (levels of at least `big` cells take the tall tiles; the simulation's
// tile_big, VT_BIG_CELLS unless the batch tuner chose otherwise)
int tile_height(unsigned nc, unsigned big) { return nc >= big ? VT_Y_BIG : VT_Y_SMALL; }

// Blocks of a tiled 2-D V-cycle kernel (vos_vcycle.h, tile_of) with tiles
// of height ty: the tile count rounded up to a multiple of the 8 XCDs.
unsigned tile_blocks(int nx, int ny, int ty)
{
  const unsigned nt = (unsigned)((nx + VT_X - 1) / VT_X) * (unsigned)((ny + ty - 1) / ty);
  return (nt + NXCD - 1) / NXCD * NXCD;
}

// Blocks of a sweep over n items: one item per thread up to MAXB blocks,
// rounded up to a multiple of the 8 XCDs (XCD-aware ranges, vos_device.h).
int grid_blocks(size_t n)
{
  size_t b = (n + TPB - 1) / TPB;
  if (b < 1) b = 1;
  if (b >= NXCD) b = (b + NXCD - 1) / NXCD * NXCD;
  if (b > (size_t)MAXB) b = MAXB;
  return (int)b;
}

struct LevelDims {
  int n[3];
  unsigned nc;
  unsigned nf[3];
  int fd[3][3];
};

LevelDims level_dims(int nx, int ny, int nz)
{
  LevelDims L;
  L.n[0] = nx; L.n[1] = ny; L.n[2] = nz;
  L.nc = (unsigned)nx * ny * nz;
  for (int d = 0; d < 3; ++d) {
    for (int e = 0; e < 3; ++e) L.fd[d][e] = L.n[e] + (e == d);
    L.nf[d] = (unsigned)L.fd[d][0] * L.fd[d][1] * L.fd[d][2];
  }
  return L;
}

// Pressure hierarchy: ceil-halve every active dimension until the level has
// <= MG_COARSE_MAX cells (the coarsest is then solved with its dense inverse).
int mg_hierarchy(const vos_grid &g, LevelDims *out)
{
  const int nd = g.nz == 1 ? 2 : 3;
  int n[3] = {g.nx, g.ny, g.nz};
  int L = 0;
  out[L++] = level_dims(n[0], n[1], n[2]);
  while (L < MG_MAX_LEVELS) {
    unsigned nc = (unsigned)n[0] * n[1] * n[2];
    if (nc <= (unsigned)MG_COARSE_MAX) break;
    for (int d = 0; d < nd; ++d) n[d] = (n[d] + 1) / 2;
    out[L++] = level_dims(n[0], n[1], n[2]);
  }
  return L;
}

constexpr int NVEC = 15;   // transport 0-10; momentum lanes 0-4, 5-9, 10-14
constexpr int NHIST = 3;  // earlier solutions kept per solve for extrapolated starts
constexpr int NSMG = 4;   // stencil hierarchies: momentum x, y, z; transport

struct SmgPlan {
  int nlev;
  int n[SMG_MAX_LEVELS][3];
  size_t off[SMG_MAX_LEVELS], diag[SMG_MAX_LEVELS], x[SMG_MAX_LEVELS], b[SMG_MAX_LEVELS], t[SMG_MAX_LEVELS];
  size_t dif[SMG_MAX_LEVELS];   // diffusive parts (transport hierarchy only)
  size_t off32[SMG_MAX_LEVELS];   // FP32 off-diagonal copies of the level (when has32)
  bool has32[SMG_MAX_LEVELS];
  bool split;
  size_t ainv;
};

struct Layout {
  size_t uprev[3][NHIST];
  size_t cprev[NHIST], pprev[NHIST];
  size_t tdiag, tdif;
  size_t eps, p, c, pn, cold, rbar, gmag, nrm[3], pdiag, off, u[3], ustar[3], dmom[3], af[3], T[3], w[3];
  size_t c0, eps_prev;   // transient storage: c at the step's start, eps at the previous step's start
  size_t vec[NVEC];
  size_t part, part2, part3, part_max, scal, ainv;
  size_t mgT[MG_MAX_LEVELS][3], mgdiag[MG_MAX_LEVELS], mgx[MG_MAX_LEVELS], mgb[MG_MAX_LEVELS], mgt[MG_MAX_LEVELS];
  int nlev;
  SmgPlan smg[NSMG];
  size_t total;
};

constexpr int NSC = 9;  // scalar blocks: mom x/y/z, pressure, transport, misc, diag, warm start, extrapolation
// Iterations without the residual halving after which a mixed-precision
// pressure solve continues with the FP64 hierarchy.
constexpr int P_STALL_WINDOW = 400;

// Aggregation hierarchy: ceil-halve every active dimension until <= SMG_COARSE_MAX cells.
void plan_smg(Plan &P, SmgPlan &S, int nx, int ny, int nz, int nd, size_t rs, bool split, bool off32 = false)
{
  int n[3] = {nx, ny, nz};
  S.nlev = 0;
  S.split = split;

  while (S.nlev < SMG_MAX_LEVELS) {
    const int l = S.nlev++;
    for (int d = 0; d < 3; ++d) S.n[l][d] = n[d];
    const size_t nc = (size_t)n[0] * n[1] * n[2];
    S.off[l] = P.take(6 * nc * rs);
    S.diag[l] = P.take(nc * rs);
    S.x[l] = P.take(nc * rs);
    S.b[l] = P.take(nc * rs);
    S.t[l] = P.take(nc * rs);
    S.dif[l] = split ? P.take(6 * nc * rs) : 0;
    // FP32 copies on the levels that run the fused legs
    S.has32[l] = off32 && zfused_level(n);
    S.off32[l] = S.has32[l] ? P.take(6 * nc * sizeof(float)) : 0;
    if (nc <= (size_t)SMG_COARSE_MAX) break;
    for (int d = 0; d < nd; ++d) n[d] = (n[d] + 1) / 2;
  }
  S.ainv = P.take((size_t)SMG_COARSE_MAX * SMG_COARSE_MAX * sizeof(double));
}

Layout make_layout(const vos_grid &g, int precision)
{
  Layout Lo;
  Plan P;
  LevelDims D0 = level_dims(g.nx, g.ny, g.nz);
  const size_t nc = D0.nc;
  const size_t dbl = sizeof(double);
  Lo.eps = P.take(nc * dbl);
  Lo.p = P.take(nc * dbl);
  Lo.c = P.take(nc * dbl);
  Lo.pn = P.take(nc * dbl);
  Lo.cold = P.take(nc * dbl);
  for (int k = 0; k < NHIST; ++k) {   // earlier steps' solutions, for extrapolated starts
    Lo.cprev[k] = P.take(nc * dbl);
    Lo.pprev[k] = P.take(nc * dbl);
  }
  Lo.rbar = P.take(nc * dbl);
  Lo.c0 = P.take(nc * dbl);
  Lo.eps_prev = P.take(nc * dbl);
  Lo.gmag = P.take(nc * dbl);
  for (int d = 0; d < 3; ++d) Lo.nrm[d] = P.take(nc * dbl);
  Lo.pdiag = P.take(nc * dbl);
  Lo.off = P.take(6 * nc * dbl);
  Lo.tdiag = P.take(nc * dbl);      // transport: diagonal and diffusive couplings of the unscaled rows
  Lo.tdif = P.take(6 * nc * dbl);
  size_t nmax = nc;
  for (int d = 0; d < 3; ++d) {
    nmax = std::max(nmax, (size_t)D0.nf[d]);
    Lo.u[d] = P.take(D0.nf[d] * dbl);
    Lo.ustar[d] = P.take(D0.nf[d] * dbl);
    Lo.dmom[d] = P.take(D0.nf[d] * dbl);
    Lo.af[d] = P.take(D0.nf[d] * dbl);
    Lo.T[d] = P.take(D0.nf[d] * dbl);
    Lo.w[d] = P.take(D0.nf[d] * dbl);
    for (int k = 0; k < NHIST; ++k) Lo.uprev[d][k] = P.take(D0.nf[d] * dbl);   // earlier predictors
  }
  for (int k = 0; k < NVEC; ++k) Lo.vec[k] = P.take(nmax * dbl);
  Lo.part = P.take((size_t)NSLOT * MAXB * dbl);
  Lo.part2 = P.take((size_t)NSLOT * MAXB * dbl);   // partials of the momentum solves on the second and third lanes
  Lo.part3 = P.take((size_t)NSLOT * MAXB * dbl);
  Lo.part_max = P.take((size_t)MAXB * dbl);
  Lo.scal = P.take((size_t)NSC * S_COUNT * 2 * dbl);
  Lo.ainv = P.take((size_t)MG_COARSE_MAX * MG_COARSE_MAX * dbl);
  LevelDims lv[MG_MAX_LEVELS];
  Lo.nlev = mg_hierarchy(g, lv);
  const size_t rs = precision == VOS_MIXED ? sizeof(float) : sizeof(double);
  // the pressure hierarchy is sized for FP64 in both modes: a mixed-precision
  // solve whose FP32 hierarchy stalls continues with an FP64 one built over it
  const size_t rsp = sizeof(double);
  for (int l = 0; l < Lo.nlev; ++l) {
    for (int d = 0; d < 3; ++d) Lo.mgT[l][d] = P.take(lv[l].nf[d] * rsp);
    Lo.mgdiag[l] = P.take(lv[l].nc * rsp);
    Lo.mgx[l] = P.take(lv[l].nc * rsp);
    Lo.mgb[l] = P.take(lv[l].nc * rsp);
    Lo.mgt[l] = P.take(lv[l].nc * rsp);
  }
  const int nd = g.nz == 1 ? 2 : 3;
  for (int d = 0; d < 3; ++d) {
    if (d < nd) plan_smg(P, Lo.smg[d], D0.fd[d][0], D0.fd[d][1], D0.fd[d][2], nd, rs, true);
    else Lo.smg[d].nlev = 0;
  }
  // the transport hierarchy is FP64 in both precisions: its Galerkin coarse
  // diagonals of upwind-dominated rows cancel to near zero and break down in
  // FP32.  In mixed precision the smoothing of its 3-D levels of >= 2^20
  // cells reads FP32 copies of their off-diagonals (FP64 arithmetic, FP64
  // diagonal, FP64 Galerkin products).
  plan_smg(P, Lo.smg[3], g.nx, g.ny, g.nz, nd, sizeof(double), true, precision == VOS_MIXED && nd == 3);
  Lo.total = P.off;
  return Lo;
}

}  // namespace

namespace vosint {
vos_status fail(vos_status st, const std::string &msg)
{
  g_err = msg;
  return st;
}
}  // namespace vosint

struct vos_sim {
  vos_grid grid;
  vos_params prm;
  vos_opts opt;
  hipStream_t stream;
  Dev g;
  Phys P;
  Layout lo;
  char *ws;
  double *eps, *p, *c, *pn, *cold, *rbar, *gmag, *nrm[3], *pdiag, *off;
  double *tdiag, *tdif;     // transport rows before scaling: diagonal, diffusive couplings
  double *c0, *eps_prev;    // transient storage: c at the step's start, eps at the previous step's start
  double *u[3], *ustar[3], *dmom[3], *af[3], *T[3], *w[3];
  double *vec[NVEC];
  double *part, *part_max, *scal, *ainv;
  int nlev;
  MgLevel<float> mgf[MG_MAX_LEVELS];
  MgLevel<double> mgd[MG_MAX_LEVELS];
  int snlev[NSMG];
  SLevel<float> smgf[NSMG][SMG_MAX_LEVELS];
  SLevel<double> smgd[NSMG][SMG_MAX_LEVELS];
  double *sainv[NSMG];
  double *host;       // pinned scalar read-back buffer
  bool solid_dt_dev;  // the last solid update took its step from the device (k_solid_dt)
  hipEvent_t ev[7];
  bool use_graphs;
  double p_scale;           // global scale of the pressure hierarchy (set per step)
  int coarse_cells;         // levels at or below this size run in the single-block kernel
  unsigned tile_big;        // 2-D tiled V-cycle legs: levels of at least this many cells take the tall tiles
  hipGraphExec_t gexec[8];  // one captured iteration chunk per solve
  int last_its[8];          // iterations the last solve of each slot took (0: none yet)

  bool have_geometry;
  bool stepped;             // a step has run: the hierarchies hold live data
  vos_diag last;

  vos_unet *net;            // attached warm-start network (or null)
  double ws_gain;
  int ws_use;
  bool ws_sampled;          // the network input of the last pressure solve is in its buffer
  double ws_s0;             // rms of the Jacobi-scaled initial residual of that solve
  int ws_used;              // the last solve started from the network's guess
  double ws_res_prev, ws_res_guess;
  double ws_drop;           // decrease of the squared A-norm error the guess achieved
  double ws_frac;           // ws_drop / squared A-norm error of starting from p^n
  int it_p_fp64;            // iterations of the last pressure solve run with the FP64 hierarchy (mixed)
  double p_res0;            // initial relative residual of the last pressure solve
  bool p_fp64_sticky;       // an FP32 pressure solve stalled on the current geometry (mixed)
  int n_cu;                 // compute units of the device (launch shapes of the fused legs)
  int nu_mom;               // sweeps per leg of the momentum hierarchies
  // extrapolated starts: the solutions of earlier steps, newest first (the host
  // rotates the buffers), and how many of them belong to the current history
  double *cprev[NHIST], *pprev[NHIST];
  int hist_c, hist_p;
  double *uprev[3][NHIST];  // earlier momentum predictors
  int hist_u[3];            // 0: no predictor of this history, 1: ustar holds one, k > 1: k - 1 earlier ones too
  // momentum and pressure hierarchies rebuilt every setup_every solves; solves since each
  // was built: 0-2 momentum, 4 pressure, 5 the mixed pressure's FP64 one after a stall
  int setup_every;
  int mg_age[6];
  // two lanes for the momentum components, each with its own stream (created back to
  // back, so they land on different hardware queues), Krylov vectors, partials and
  // pinned read-back buffer; component 1 is driven from a second host thread
  hipStream_t lane_stream[3];   // momentum lanes (the third in 3-D only)
  double *part2, *part3;        // block partials of lanes 1 and 2
  double *host2, *host3;        // pinned read-back buffers of lanes 1 and 2
  hipEvent_t fork, join[3];
};

namespace {

double *sc_block(vos_sim *s, int k) { return s->scal + (size_t)k * S_COUNT * 2; }
enum { SC_MOM = 0, SC_P = 3, SC_C = 4, SC_MISC = 5, SC_DIAG = 6, SC_WS = 7, SC_EX = 8 };
enum { H_MOM = 0, H_P = 4, H_P64 = 5 };

// Whether hierarchy h is rebuilt for this solve (it is once setup_every solves
// have used it, and after any state change); counts the solve.
bool hierarchy_due(vos_sim *s, int h)
{
  const bool due = s->mg_age[h] >= s->setup_every;
  s->mg_age[h] = due ? 1 : s->mg_age[h] + 1;
  return due;
}

void hierarchies_stale(vos_sim *s)
{
  for (int h = 0; h < 6; ++h) s->mg_age[h] = 1 << 30;
}

template <typename R>
void fill_levels(vos_sim *s, MgLevel<R> *lv)
{
  const vos_grid &g = s->grid;
  LevelDims ld[MG_MAX_LEVELS];
  int nl = mg_hierarchy(g, ld);
  for (int l = 0; l < nl; ++l) {
    MgLevel<R> &L = lv[l];
    for (int d = 0; d < 3; ++d) {
      L.n[d] = ld[l].n[d];
      L.nf[d] = ld[l].nf[d];
      for (int e = 0; e < 3; ++e) L.fd[d][e] = ld[l].fd[d][e];
      L.T[d] = (R *)(s->ws + s->lo.mgT[l][d]);
    }
    L.nc = ld[l].nc;
    L.dsum = l == 0;   // k_mg_diag builds the finest diagonal from the faces
    L.diag = (R *)(s->ws + s->lo.mgdiag[l]);
    L.x = (R *)(s->ws + s->lo.mgx[l]);
    L.b = (R *)(s->ws + s->lo.mgb[l]);
    L.t = (R *)(s->ws + s->lo.mgt[l]);
  }
}

template <typename R>
void fill_smg(vos_sim *s, int h, SLevel<R> *lv)
{
  const SmgPlan &S = s->lo.smg[h];
  s->snlev[h] = S.nlev;
  for (int l = 0; l < S.nlev; ++l) {
    SLevel<R> &L = lv[l];
    for (int d = 0; d < 3; ++d) L.n[d] = S.n[l][d];
    L.nc = (unsigned)L.n[0] * L.n[1] * L.n[2];
    L.off = (R *)(s->ws + S.off[l]);
    L.diag = (R *)(s->ws + S.diag[l]);
    L.x = (R *)(s->ws + S.x[l]);
    L.b = (R *)(s->ws + S.b[l]);
    L.t = (R *)(s->ws + S.t[l]);
    L.dif = S.split ? (R *)(s->ws + S.dif[l]) : nullptr;
    // the 3-D transport level 0's diffusive parts are the assembly's own
    if constexpr (std::is_same<R, double>::value)
      if (h == 3 && l == 0 && s->g.nd == 3) L.dif = s->tdif;
    L.off32 = S.has32[l] ? (float *)(s->ws + S.off32[l]) : nullptr;
  }
  if (S.nlev) s->sainv[h] = (double *)(s->ws + S.ainv);
}

vos_status check_grid(const vos_grid *g)
{
  if (!g) return fail(VOS_ERR_ARG, "grid is NULL");
  if (g->nx < 2 || g->ny < 1 || g->nz < 1 || !(g->dx > 0.0))
    return fail(VOS_ERR_ARG, "grid needs nx >= 2, ny >= 1, nz >= 1, dx > 0");
  if ((double)g->nx * g->ny * g->nz > 2.0e9 || (double)(g->nx + 1) * g->ny * g->nz > 2.0e9)
    return fail(VOS_ERR_ARG, "grid too large for 32-bit indexing");
  return VOS_OK;
}

vos_status check_opts(const vos_opts *o)
{
  if (!o) return fail(VOS_ERR_ARG, "opts is NULL");
  if (!(o->rtol_u > 0) || !(o->rtol_p > 0) || !(o->rtol_c > 0)) return fail(VOS_ERR_ARG, "tolerances must be > 0");
  if (o->maxit_u < 1 || o->maxit_p < 1 || o->maxit_c < 1) return fail(VOS_ERR_ARG, "maxit must be >= 1");
  if (o->precision != VOS_FP64 && o->precision != VOS_MIXED) return fail(VOS_ERR_ARG, "unknown precision");
  if (o->mg_nu < 0 || o->mg_nu > 8) return fail(VOS_ERR_ARG, "mg_nu must be in [0, 8]");
  if (o->check_every < 1 || o->check_every > 256) return fail(VOS_ERR_ARG, "check_every must be in [1, 256]");
  if (o->coarse_cells != 0 && (o->coarse_cells < 64 || o->coarse_cells > 65536))
    return fail(VOS_ERR_ARG, "coarse_cells must be 0 or in [64, 65536]");
  if (o->level_kernels != 0 && o->level_kernels != 1) return fail(VOS_ERR_ARG, "level_kernels must be 0 or 1");
  if (o->p_fp32_its < 0) return fail(VOS_ERR_ARG, "p_fp32_its must be >= 0");
  if (o->extrapolate < 0 || o->extrapolate > 2) return fail(VOS_ERR_ARG, "extrapolate must be 0, 1 or 2");
  if (o->setup_every < 0 || o->setup_every > 1000) return fail(VOS_ERR_ARG, "setup_every must be in [0, 1000]");
  if (!(o->deps_max >= 0.0) || !std::isfinite(o->deps_max))
    return fail(VOS_ERR_ARG, "deps_max must be finite and >= 0");
  if (!(o->solid_dt >= 0.0) || !std::isfinite(o->solid_dt))
    return fail(VOS_ERR_ARG, "solid_dt must be finite and >= 0");
  if (o->simple != 0 && o->simple != 1) return fail(VOS_ERR_ARG, "simple must be 0 or 1");
  if (o->simple) {
    if (o->outer_max < 1) return fail(VOS_ERR_ARG, "outer_max must be >= 1");
    if (!(o->outer_tol >= 0.0) || !std::isfinite(o->outer_tol)) return fail(VOS_ERR_ARG, "outer_tol must be >= 0");
    if (!(o->relax_u > 0.0 && o->relax_u <= 1.0) || !(o->relax_p > 0.0 && o->relax_p <= 1.0) ||
        !(o->relax_c > 0.0 && o->relax_c <= 1.0))
      return fail(VOS_ERR_ARG, "relaxation factors must be in (0, 1]");
    if (o->extrapolate) return fail(VOS_ERR_ARG, "extrapolated starts belong to the one-pass step (simple = 0)");
  }
  return VOS_OK;
}

vos_status check_params(const vos_params *p)
{
  if (!p) return fail(VOS_ERR_ARG, "params is NULL");
  if (!(p->mu > 0) || !(p->rho > 0) || !(p->k0 > 0) || !(p->D >= 0) || !(p->kc >= 0) || !(p->Vm >= 0) ||
      !(p->zeta >= 0) || !(p->eps_min > 0 && p->eps_min < 1) || !(p->u_in >= 0))
    return fail(VOS_ERR_ARG, "physical parameters out of range");
  if (p->model < 0 || p->model > 2) return fail(VOS_ERR_ARG, "unknown model");
  if (p->drive != 0 && p->drive != 1) return fail(VOS_ERR_ARG, "drive must be 0 (velocity) or 1 (pressure)");
  if (!std::isfinite(p->p_in) || !std::isfinite(p->p_out)) return fail(VOS_ERR_ARG, "pressures must be finite");
  if (p->convection != 0 && p->convection != 1) return fail(VOS_ERR_ARG, "convection must be 0 or 1");
  if (p->grad_scheme != 0 && p->grad_scheme != 1) return fail(VOS_ERR_ARG, "grad_scheme must be 0 or 1");
  if (p->grad_scheme == 1 && p->model == VOS_IVOS)
    return fail(VOS_ERR_ARG, "the decentred gradient is a VoS-psi variant (iVoS keeps its central normals)");
  if (p->psi_kind != 0 && p->psi_kind != 1) return fail(VOS_ERR_ARG, "psi_kind must be 0 or 1");
  if (p->psi_kind == 1 && p->model == VOS_PSI_PRIME)
    return fail(VOS_ERR_ARG, "VoS-psi' fits lambda to eps (1 - eps): psi = 1 is for VoS-psi");
  if (p->transient != 0 && p->transient != 1) return fail(VOS_ERR_ARG, "transient must be 0 or 1");
  if (!(p->Vm_f >= 0.0) || !std::isfinite(p->Vm_f)) return fail(VOS_ERR_ARG, "Vm_f must be finite and >= 0");
  return VOS_OK;
}

// Compute units of the current device (256 if the query fails).
int device_cus()
{
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n < 1)
    n = 256;
  return n;
}

// Options that do not go with some parameters.
vos_status check_combination(const vos_params *p, const vos_opts *o)
{
  if (o->solid_dt > 0.0 && p->transient)
    return fail(VOS_ERR_ARG, "solid_dt separates the solid step from dt, which the transient storage terms take");
  return VOS_OK;
}

// The solid update's step before the deps_max bound: solid_dt when set, else dt.
double solid_nominal(const vos_sim *s, double dt);

// Device copy of the physical parameters (and the SIMPLE relaxations the kernels apply).
void fill_phys(Phys &P, const vos_params *params, const vos_opts &o)
{
  P.mu = params->mu; P.rho = params->rho; P.D = params->D; P.k0 = params->k0; P.kc = params->kc;
  P.Vm = params->Vm; P.zeta = params->zeta; P.c_in = params->c_in; P.eps_min = params->eps_min;
  P.u_in = params->u_in; P.p_out = params->p_out; P.model = params->model;
  P.p_in = params->p_in; P.convection = params->convection; P.grad_scheme = params->grad_scheme;
  P.psi_kind = params->psi_kind; P.transient = params->transient; P.Vm_f = params->Vm_f;
  P.simple = o.simple;
  P.relax_u = o.simple ? o.relax_u : 1.0;
  P.relax_c = o.simple ? o.relax_c : 1.0;
}

// Host read of n doubles from device memory (synchronises the stream).
// Where a solve runs: its stream, Krylov vectors, block partials and pinned
// read-back buffer.  The main lane is the sim's own; the second lane lets a
// momentum component run concurrently with another.
struct Lane {
  hipStream_t st;
  double *const *vec;
  double *part;
  double *host;
};

Lane main_lane(vos_sim *s) { return Lane{s->stream, s->vec, s->part, s->host}; }
Lane momentum_lane(vos_sim *s, int k)
{
  if (k == 0) return Lane{s->lane_stream[0], s->vec, s->part, s->host};
  if (k == 1) return Lane{s->lane_stream[1], s->vec + 5, s->part2, s->host2};
  return Lane{s->lane_stream[2], s->vec + 10, s->part3, s->host3};
}

vos_status read_back(const Lane &ln, const double *dev, size_t n)
{
  HIP_TRY(hipMemcpyAsync(ln.host, dev, n * sizeof(double), hipMemcpyDeviceToHost, ln.st));
  HIP_TRY(hipStreamSynchronize(ln.st));
  return VOS_OK;
}

vos_status read_back(vos_sim *s, const double *dev, size_t n) { return read_back(main_lane(s), dev, n); }

// Run iterations until the device flag says converged or maxit is reached.
// With graphs on, a chunk of check_every iterations is captured once per
// solve (gid) and replayed; every kernel in it returns at once after the flag
// is set, so replaying a whole chunk past convergence changes nothing.  The
// first host check comes after as many whole chunks as fit in the iterations
// the last solve of the same slot took, later checks after every chunk.
// Stall rule of a solve that may switch preconditioners: give up once the
// residual has not halved within `window` iterations, or after `cap`
// iterations (0: no cap).  window 0: never.
struct Stall {
  int window = 0, cap = 0;
  bool hit = false, by_cap = false;
};

template <typename F>
vos_status krylov_loop(vos_sim *s, const Lane &ln, int gid, double *sc, int maxit, F &&iter, int *its, double *res2,
                       double *tol2, bool *conv, Stall *stall = nullptr)
{
  HIP_TRY(hipGetLastError());
  int launched = 0;
  const double *host = ln.host;
  vos_status st = VOS_OK;
  // no read-back before the first chunk: when the start already meets the
  // tolerance every kernel of the chunk finds the device flag set and returns
  bool done = false;
  const int chunk = s->opt.check_every;
  double mark = HUGE_VAL;
  int mark_its = 0;
  // one chunk of iterations: a replay of the captured graph, or plain launches
  auto launch_chunk = [&]() -> vos_status {
    if (s->use_graphs) {
      if (!s->gexec[gid]) {
        hipGraph_t graph;
        HIP_TRY(hipStreamBeginCapture(ln.st, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < chunk; ++i) iter();
        hipError_t e = hipStreamEndCapture(ln.st, &graph);
        if (e != hipSuccess) return fail(VOS_ERR_DEVICE, std::string("graph capture: ") + hipGetErrorString(e));
        e = hipGraphInstantiate(&s->gexec[gid], graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        if (e != hipSuccess) { s->gexec[gid] = nullptr; return fail(VOS_ERR_DEVICE, "hipGraphInstantiate failed"); }
      }
      HIP_TRY(hipGraphLaunch(s->gexec[gid], ln.st));
      launched += chunk;
    } else {
      const int k = std::min(chunk, maxit - launched);
      for (int i = 0; i < k; ++i) iter();
      launched += k;
    }
    return VOS_OK;
  };
  int ahead = std::max(1, s->last_its[gid] / chunk);
  while (!done && launched < maxit) {
    for (int a = 0; a < ahead && launched < maxit; ++a)
      if (vos_status e = launch_chunk()) return e;
    ahead = 1;
    HIP_TRY(hipGetLastError());
    st = read_back(ln, sc, S_COUNT);
    if (st) return st;
    done = host[S_CONV] != 0.0;
    if (stall && !done) {
      const int it = (int)host[S_ITS];
      if (host[S_RES2] <= 0.25 * mark) {
        mark = host[S_RES2];
        mark_its = it;
      }
      const bool capped = stall->cap > 0 && it >= stall->cap;
      if (capped || (stall->window > 0 && it - mark_its >= stall->window)) {
        stall->hit = true;
        stall->by_cap = capped;
        break;
      }
    }
  }
  *its = (int)host[S_ITS];
  s->last_its[gid] = *its;
  *res2 = host[S_RES2];
  *tol2 = host[S_TOL2];
  *conv = (host[S_RES2] <= host[S_TOL2]) || (host[S_RES2] == 0.0);
  return VOS_OK;
}

void drop_graphs(vos_sim *s)
{
  for (int k = 0; k < 8; ++k)
    if (s->gexec[k]) { (void)hipGraphExecDestroy(s->gexec[k]); s->gexec[k] = nullptr; }
}

// Start of a solve from the linear extrapolation in time of the last two
// solutions: x = 2 x^n - x^(n-1) when have_prev, and prev = x^n either way.
// Start of the next solve from x = x^n and the earlier solutions h[0] =
// x^(n-1), h[1] = x^(n-2), h[2] = x^(n-3), hist of them valid: x^n (hist 0),
// the linear extrapolation 2 x^n - x^(n-1), or, when quad is allowed and the
// flag says the quadratic one predicted x^n better, 3 x^n - 3 x^(n-1) +
// x^(n-2).  Partials: squared errors of the linear (hist >= 2) and quadratic
// (hist >= 3) predictions of x^n.  x^n is stored over h[2], the buffer the
// host then rotates to the front.
__global__ void __launch_bounds__(TPB) k_extrap(unsigned n, int hist, int quad_ok, const double *__restrict__ flag,
                                                double *__restrict__ x, const double *__restrict__ h0,
                                                const double *__restrict__ h1, double *__restrict__ h2,
                                                double *__restrict__ part)
{
  const bool quad = quad_ok && hist >= 2 && flag[0] != 0.0;
  double e1 = 0.0, e2 = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double xn = x[i], a = h0[i], b = h1[i], c = h2[i];
    double st = xn;
    if (hist >= 1) st = quad ? 3.0 * xn - 3.0 * a + b : 2.0 * xn - a;
    x[i] = st;
    h2[i] = xn;
    if (hist >= 2) {
      const double d = xn - (2.0 * a - b);
      e1 += d * d;
    }
    if (hist >= 3) {
      const double d = xn - (3.0 * a - 3.0 * b + c);
      e2 += d * d;
    }
  }
  const double v[2] = {e1, e2};
  write_partials<2>(v, part);
}

// The order of the next extrapolated start: quadratic (flag 1) when it
// predicted the newest solution better than the linear one did.
__global__ void k_extrap_order(const double *__restrict__ part, int nb, int hist, double *__restrict__ flag)
{
  const double e1 = sum_partials(part, 0, nb);
  const double e2 = sum_partials(part, 1, nb);
  if (threadIdx.x == 0) flag[0] = (hist >= 3 && e2 < e1) ? 1.0 : 0.0;
}

// Extrapolated start of x over the history h (hist valid entries, newest
// first); rotates h so that h[0] = the old x; *hist grows to at most NHIST.
// Slot f of the extrapolation scalar block keeps the order chosen for field f.
void extrapolate(vos_sim *s, hipStream_t st, double *part, unsigned n, double *x, double **h, int *hist, int f)
{
  const int nb = grid_blocks(n);
  double *flag = sc_block(s, SC_EX) + f;
  const int quad = s->opt.extrapolate == 2;
  k_extrap<<<nb, TPB, 0, st>>>(n, *hist, quad, flag, x, h[0], h[1], h[2], part);
  if (quad) k_extrap_order<<<1, TPB, 0, st>>>(part, nb, *hist, flag);
  double *t = h[2];
  h[2] = h[1];
  h[1] = h[0];
  h[0] = t;
  *hist = std::min(NHIST, *hist + 1);
}

// q = A x (pressure operator) with the partials of x.q in s->part; returns
// the number of partial blocks.
int p_apply(vos_sim *s, const double *x, double *q, const double *flag)
{
  const Dev &g = s->g;
  if (papply_marching(g)) {
    const int zl = papply_zlen(g);
    const unsigned nb = zrun_blocks(g.n, zl);
    k_p_apply3d<<<nb, TPB, 0, s->stream>>>(g, s->T[0], s->T[1], s->T[2], x, q, s->part, zl, flag);
    return (int)nb;
  }
  const int nb = grid_blocks(g.nc);
  k_p_apply<<<nb, TPB, 0, s->stream>>>(g, s->T[0], s->T[1], s->T[2], x, q, s->part, flag);
  return nb;
}

// ---------------------------------------------------------------- stage S1

void launch_coefficients(vos_sim *s, double dt)
{
  const Dev &g = s->g;
  hipStream_t st = s->stream;
  k_face_coef<0><<<grid_blocks(g.nf[0]), TPB, 0, st>>>(g, s->P, dt, s->eps, s->dmom[0], s->af[0], s->T[0]);
  k_face_coef<1><<<grid_blocks(g.nf[1]), TPB, 0, st>>>(g, s->P, dt, s->eps, s->dmom[1], s->af[1], s->T[1]);
  if (g.nd == 3)
    k_face_coef<2><<<grid_blocks(g.nf[2]), TPB, 0, st>>>(g, s->P, dt, s->eps, s->dmom[2], s->af[2], s->T[2]);
  const int nb = grid_blocks(g.nc);
  k_cell_grad<<<nb, TPB, 0, st>>>(g, s->P.grad_scheme, s->eps, s->gmag, s->nrm[0], s->nrm[1], s->nrm[2], s->part);
  k_lambda<<<1, TPB, 0, st>>>(s->part, nb, s->P.model, sc_block(s, SC_MISC));
  k_face_w<0><<<grid_blocks(g.nf[0]), TPB, 0, st>>>(g, s->P.kc, s->nrm[0], s->w[0]);
  k_face_w<1><<<grid_blocks(g.nf[1]), TPB, 0, st>>>(g, s->P.kc, s->nrm[1], s->w[1]);
  if (g.nd == 3) k_face_w<2><<<grid_blocks(g.nf[2]), TPB, 0, st>>>(g, s->P.kc, s->nrm[2], s->w[2]);
  k_pdiag<<<nb, TPB, 0, st>>>(g, s->T[0], s->T[1], s->T[2], s->pdiag);
}

// ---------------------------------------------------------------- algorithmic bytes
// Each array read or written once per launch (neighbour re-reads come from
// cache and are not counted).  R = arithmetic of the hierarchy.  Finest-level
// Jacobi sweep on an explicit stencil: read x, b, diag and 2nd off-diagonals,
// write x (+ the FP64 result on the last sweep).
template <typename R>
double jacobi_bytes(unsigned nc, int nd, bool out64, bool finest)
{
  (void)finest;
  return ((4.0 + 2 * nd) * sizeof(R) + (out64 ? 8.0 : 0.0)) * nc;
}

// ---------------------------------------------------------------- stencil multigrid

// Coarse levels and coarsest inverse of hierarchy h (level 0 already filled).
template <typename R>
void smg_coarsen_all(vos_sim *s, int h, SLevel<R> *lv, hipStream_t st)
{
  const int nd = s->g.nd;
  const int L = s->snlev[h];
  for (int l = 0; l + 1 < L; ++l) {
    const dim3 gr(grid_blocks(lv[l + 1].nc));
    if (l == 0 && h == 3 && lv[0].off32) {   // level 0's FP64 off-diagonals formed from the assembly
      if (nd == 3) k_smg_coarsen<R, 3, true><<<gr, TPB, 0, st>>>(lv[0], lv[1], s->off, s->tdiag);
      else k_smg_coarsen<R, 2, true><<<gr, TPB, 0, st>>>(lv[0], lv[1], s->off, s->tdiag);
    } else if (nd == 3) {
      k_smg_coarsen<R, 3><<<gr, TPB, 0, st>>>(lv[l], lv[l + 1]);
    } else {
      k_smg_coarsen<R, 2><<<gr, TPB, 0, st>>>(lv[l], lv[l + 1]);
    }
  }
  k_smg_coarse_inverse<R><<<1, GJ_TPB, 0, st>>>(lv[L - 1], nd, s->sainv[h]);
}

// Cells per thread on the first level of a coarse tail (levels lc..L-1) that
// runs in LDS (k_v_coarse_lds): 1, 2 or (FP32) 4 -- an FP64 tail with 4 would
// spill registers; 0 when the tail does not qualify (not 2-D, first level
// above that many cells per thread, a later level above one cell per thread,
// or more than VCL_CELLS cells in all).
template <typename Lv>
int coarse_in_lds(const Lv *lv, int lc, int L, int nd, bool fused)
{
  if (!fused || nd != 2 || L - lc > VCL_MAXLV) return 0;
  const unsigned c0max = sizeof(*lv[0].x) == 8 ? 2u : (unsigned)VCL_C0;
  unsigned tot = 0;
  for (int l = lc; l < L; ++l) {
    const unsigned cap = (unsigned)VC_COARSE_TPB * (l == lc ? c0max : 1u);
    if (lv[l].nc > cap) return 0;
    tot += lv[l].nc;
  }
  if (tot > (unsigned)VCL_CELLS) return 0;
  const unsigned c0 = (lv[lc].nc + VC_COARSE_TPB - 1) / VC_COARSE_TPB;
  return c0 <= 1 ? 1 : (c0 <= 2 ? 2 : 4);
}

template <typename Lv, typename R>
void launch_coarse(int c0, const LevelPack<Lv> &pack, int lc, int L, int nd, int nu, R om, const double *Ainv,
                   const double *sc, hipStream_t st)
{
  if (c0 == 1) k_v_coarse_lds<Lv, R, 1><<<1, VC_COARSE_TPB, 0, st>>>(pack, lc, L, nu, om, Ainv, sc);
  else if (c0 == 2) k_v_coarse_lds<Lv, R, 2><<<1, VC_COARSE_TPB, 0, st>>>(pack, lc, L, nu, om, Ainv, sc);
  else if (sizeof(R) == 4 && c0 == 4) k_v_coarse_lds<Lv, R, sizeof(R) == 4 ? 4 : 2><<<1, VC_COARSE_TPB, 0, st>>>(
      pack, lc, L, nu, om, Ainv, sc);
  else k_v_coarse_cycle<Lv, R><<<1, VC_COARSE_TPB, 0, st>>>(pack, lc, L, nd, nu, om, Ainv, sc);
}

// Blocks a CU holds at once of the fused legs of one level type (their LDS and
// registers decide it; queried once per instantiation), times the CUs.
template <typename Lv, typename R, bool O32>
int fused_slots(const vos_sim *s)
{
  // kernel attributes: the same for every simulation of the process; the
  // initialisation of a function-local static is thread-safe (the momentum
  // lanes reach it from their own host threads)
  static const int per_cu = []() {
    int a = 0, b = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &a, reinterpret_cast<const void *>(k_v_down3d<Lv, R, RHS_R, O32>), ZT_X * zf_rows<R>, 0) != hipSuccess ||
        a < 1)
      a = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &b, reinterpret_cast<const void *>(k_v_up3d<Lv, R, true, O32>), ZT_X * zf_rows<R>, 0) != hipSuccess ||
        b < 1)
      b = 1;
    return std::min(a, b);
  }();
  return s->n_cu * per_cu;
}

// Only the FP64 aggregation levels carry FP32 off-diagonal copies (the finest
// transport level in mixed precision); the fused legs' O32 variant exists for them.
template <typename Lv>
constexpr bool lv_can32 = false;
template <>
constexpr bool lv_can32<SLevel<double>> = true;
template <typename Lv>
bool lv_has32(const Lv &)
{
  return false;
}
template <typename R>
bool lv_has32(const SLevel<R> &L)
{
  return L.off32 != nullptr;
}

// The fused legs of level F (coarse level C): the down leg from the FP64
// residual r (finest level, RHS_R) or from F's b; the up leg into the FP64
// output z (finest level) or into F.t.
// rg: the finest level's input is r times its diagonal (RHS_RG); only the
// FP64 aggregation levels (the transport hierarchy) take it.
template <typename Lv, typename R, bool O32>
void fused_down_t(vos_sim *s, const Lv &F, const Lv &C, bool finest, const double *r, double rscale, R om,
                  const double *sc, hipStream_t st, bool rg)
{
  constexpr int FY = zf_rows<R>, TPB_F = ZT_X * FY;
  const int zl = zrun_len_fused(F.n, fused_slots<Lv, R, O32>(s), FY);
  const dim3 gr(zrun_blocks_fused(F.n, zl, FY));
  if constexpr (lv_can32<Lv>) {
    if (finest && rg) return (void)(k_v_down3d<Lv, R, RHS_RG, O32><<<gr, TPB_F, 0, st>>>(F, C, r, 1.0, om, zl, sc));
  }
  if (finest) k_v_down3d<Lv, R, RHS_R, O32><<<gr, TPB_F, 0, st>>>(F, C, r, rscale, om, zl, sc);
  else k_v_down3d<Lv, R, RHS_B, O32><<<gr, TPB_F, 0, st>>>(F, C, r, rscale, om, zl, sc);
}
template <typename Lv, typename R, bool O32>
void fused_up_t(vos_sim *s, const Lv &F, const Lv &C, bool finest, double *z, const double *r, double rscale, R om,
                const double *sc, hipStream_t st, bool rg)
{
  constexpr int FY = zf_rows<R>, TPB_F = ZT_X * FY;
  const int zl = zrun_len_fused(F.n, fused_slots<Lv, R, O32>(s), FY);
  const dim3 gr(zrun_blocks_fused(F.n, zl, FY));
  if constexpr (lv_can32<Lv>) {
    if (finest && rg)
      return (void)(k_v_up3d<Lv, R, true, O32, true><<<gr, TPB_F, 0, st>>>(F, C, F.t, om, z, nullptr, r, 1.0, zl,
                                                                              sc));
  }
  if (finest) k_v_up3d<Lv, R, true, O32><<<gr, TPB_F, 0, st>>>(F, C, F.t, om, z, nullptr, r, rscale, zl, sc);
  else k_v_up3d<Lv, R, false, O32><<<gr, TPB_F, 0, st>>>(F, C, F.t, om, nullptr, nullptr, nullptr, 1.0, zl, sc);
}
template <typename Lv, typename R>
void fused_down(vos_sim *s, const Lv &F, const Lv &C, bool finest, const double *r, double rscale, R om,
                const double *sc, hipStream_t st, bool rg = false)
{
  if constexpr (lv_can32<Lv>) {
    if (lv_has32(F)) return fused_down_t<Lv, R, true>(s, F, C, finest, r, rscale, om, sc, st, rg);
  }
  fused_down_t<Lv, R, false>(s, F, C, finest, r, rscale, om, sc, st, rg);
}
template <typename Lv, typename R>
void fused_up(vos_sim *s, const Lv &F, const Lv &C, bool finest, double *z, const double *r, double rscale, R om,
              const double *sc, hipStream_t st, bool rg = false)
{
  if constexpr (lv_can32<Lv>) {
    if (lv_has32(F)) return fused_up_t<Lv, R, true>(s, F, C, finest, z, r, rscale, om, sc, st, rg);
  }
  fused_up_t<Lv, R, false>(s, F, C, finest, z, r, rscale, om, sc, st, rg);
}

// First level of a hierarchy's coarse tail (the levels of at most coarse_cells).
template <typename Lv>
int coarse_start(const vos_sim *s, const Lv *lv, int L)
{
  int lc = 0;
  while (lc < L - 1 && lv[lc].nc > (unsigned)s->coarse_cells) ++lc;
  return lc;
}

// Level F of a V-cycle with nu sweeps a leg runs the fused 3-D legs.
template <typename Lv>
bool fused_level(const vos_sim *s, const Lv &F, int nu, const double *dsc)
{
  return s->opt.level_kernels == 0 && s->g.nd == 3 && F.n[0] >= ZT_X / 2 && F.n[1] >= 2 && F.n[2] >= 2 && nu == 2 &&
         !dsc && zfused_level(F.n);
}

// z = V-cycle(r) on a hierarchy of L levels (generic over the level type).
// rg: the input is r d with d the finest level's diagonal, formed by the
// finest level's fused legs from r (callers pass it only where
// fused_level holds for that level, which precedes the coarse tail).
template <typename Lv, typename R>
void vcycle(vos_sim *s, Lv *lv, int L, const double *Ainv, const double *r, double *z, const double *sc,
            double omega, const double *dsc, double rscale, int nu, hipStream_t st, bool rg = false)
{
  const int nd = s->g.nd;
  const R om = (R)omega;
  const int lc = coarse_start(s, lv, L);
  const bool fused = s->opt.level_kernels == 0;
  // 2-D levels with 2..4 sweeps each way: one tiled kernel per leg (vos_vcycle.h)
  auto tiled = [&](const Lv &F) { return fused && nd == 2 && nu >= 2 && nu <= 4 && F.n[0] >= 2 && F.n[1] >= 2; };
  auto tgrid = [&](const Lv &F) { return dim3(tile_blocks(F.n[0], F.n[1], tile_height(F.nc, s->tile_big))); };
  // 3-D levels at least half a tile wide: z-marching kernels (vos_march3d.h)
  auto zmarch = [&](const Lv &F) { return fused && nd == 3 && F.n[0] >= ZT_X / 2 && F.n[1] >= 2 && F.n[2] >= 2; };
  for (int l = 0; l < lc; ++l) {
    Lv &F = lv[l];
    const int nb = grid_blocks(F.nc);
    if (fused_level(s, F, nu, dsc)) {
      // both pre-sweeps and the restriction in one march
      fused_down<Lv, R>(s, F, lv[l + 1], l == 0, r, rscale, om, sc, st, rg && l == 0);
      continue;
    }
    if (zmarch(F)) {
      const int zl = zrun_len(F.n);
      const dim3 gr(zrun_blocks(F.n, zl));
      if (nu == 1) {
        if (l == 0) k_v_pre<Lv, R, true, 1><<<nb, TPB, 0, st>>>(F, nd, r, dsc, rscale, om, sc);
        else k_v_pre<Lv, R, false, 1><<<nb, TPB, 0, st>>>(F, nd, r, dsc, rscale, om, sc);
      } else {
        if (l > 0) k_v_pre3d<Lv, R, RHS_B><<<gr, TPB, 0, st>>>(F, r, dsc, rscale, om, zl, sc);
        else if (dsc) k_v_pre3d<Lv, R, RHS_RD><<<gr, TPB, 0, st>>>(F, r, dsc, rscale, om, zl, sc);
        else k_v_pre3d<Lv, R, RHS_R><<<gr, TPB, 0, st>>>(F, r, dsc, rscale, om, zl, sc);
      }
      for (int k = 2; k < nu; ++k) {
        k_v_jacobi3d<Lv, R, false><<<gr, TPB, 0, st>>>(F, F.x, F.t, om, nullptr, nullptr, zl, sc);
        std::swap(F.x, F.t);
      }
      k_v_restrict3d<Lv, R><<<gr, TPB, 0, st>>>(F, lv[l + 1], zl, sc);
      continue;
    }
    if (tiled(F)) {
      const dim3 gr = tgrid(F);
#define VDOWN(NU_, TY_)                                                                                   \
  if (l == 0) k_v_down2d<Lv, R, true, NU_, TY_><<<gr, TPB, 0, st>>>(F, lv[l + 1], r, dsc, rscale, om, sc); \
  else k_v_down2d<Lv, R, false, NU_, TY_><<<gr, TPB, 0, st>>>(F, lv[l + 1], r, dsc, rscale, om, sc);
      if (tile_height(F.nc, s->tile_big) == VT_Y_BIG) {
        if (nu == 2) { VDOWN(2, VT_Y_BIG) } else if (nu == 3) { VDOWN(3, VT_Y_BIG) } else { VDOWN(4, VT_Y_BIG) }
      } else {
        if (nu == 2) { VDOWN(2, VT_Y_SMALL) } else if (nu == 3) { VDOWN(3, VT_Y_SMALL) } else { VDOWN(4, VT_Y_SMALL) }
      }
#undef VDOWN
      continue;
    }
    {
      if (nu == 1) {
        if (l == 0) k_v_pre<Lv, R, true, 1><<<nb, TPB, 0, st>>>(F, nd, r, dsc, rscale, om, sc);
        else k_v_pre<Lv, R, false, 1><<<nb, TPB, 0, st>>>(F, nd, r, dsc, rscale, om, sc);
      } else {
        if (l == 0) k_v_pre<Lv, R, true, 2><<<nb, TPB, 0, st>>>(F, nd, r, dsc, rscale, om, sc);
        else k_v_pre<Lv, R, false, 2><<<nb, TPB, 0, st>>>(F, nd, r, dsc, rscale, om, sc);
      }
    }
    for (int k = 2; k < nu; ++k) {
      k_v_jacobi<Lv, R, false><<<nb, TPB, 0, st>>>(F, nd, F.x, F.t, om, nullptr, nullptr, sc);
      std::swap(F.x, F.t);
    }
    k_v_restrict<Lv, R><<<grid_blocks(lv[l + 1].nc), TPB, 0, st>>>(F, lv[l + 1], nd, sc);
  }
  LevelPack<Lv> pack;
  for (int l = 0; l < L && l < VC_MAX_LEVELS; ++l) pack.lv[l] = lv[l];
  if (lc == 0) k_v_cast_in<Lv, R><<<grid_blocks(lv[0].nc), TPB, 0, st>>>(lv[0], r, dsc, rscale, sc);
  launch_coarse<Lv, R>(coarse_in_lds(lv, lc, L, nd, fused), pack, lc, L, nd, nu, om, Ainv, sc, st);
  if (lc == 0) {
    k_v_cast_out<Lv, R><<<grid_blocks(lv[0].nc), TPB, 0, st>>>(lv[0], z, dsc, sc);
    return;
  }
  for (int l = lc - 1; l >= 0; --l) {
    Lv &F = lv[l];
    const int nb = grid_blocks(F.nc);
    if (fused_level(s, F, nu, dsc)) {
      // prolongation and both post-sweeps in one march
      fused_up<Lv, R>(s, F, lv[l + 1], l == 0, z, r, rscale, om, sc, st, rg && l == 0);
      if (l > 0) std::swap(F.x, F.t);
      continue;
    }
    if (zmarch(F)) {
      const int zl = zrun_len(F.n);
      const dim3 gr(zrun_blocks(F.n, zl));
      if (l == 0 && nu == 1) k_v_post3d<Lv, R, true><<<gr, TPB, 0, st>>>(F, lv[l + 1], F.t, om, z, dsc, zl, sc);
      else k_v_post3d<Lv, R, false><<<gr, TPB, 0, st>>>(F, lv[l + 1], F.t, om, nullptr, nullptr, zl, sc);
      std::swap(F.x, F.t);
      for (int k = 1; k < nu; ++k) {
        if (l == 0 && k == nu - 1) k_v_jacobi3d<Lv, R, true><<<gr, TPB, 0, st>>>(F, F.x, F.t, om, z, dsc, zl, sc);
        else k_v_jacobi3d<Lv, R, false><<<gr, TPB, 0, st>>>(F, F.x, F.t, om, nullptr, nullptr, zl, sc);
        std::swap(F.x, F.t);
      }
      continue;
    }
    if (tiled(F)) {
      const dim3 gr = tgrid(F);
#define VUP(NU_, TY_)                                                                                      \
  if (l == 0) k_v_up2d<Lv, R, true, NU_, TY_><<<gr, TPB, 0, st>>>(F, lv[l + 1], F.t, om, z, dsc, sc);       \
  else k_v_up2d<Lv, R, false, NU_, TY_><<<gr, TPB, 0, st>>>(F, lv[l + 1], F.t, om, nullptr, nullptr, sc);
      if (tile_height(F.nc, s->tile_big) == VT_Y_BIG) {
        if (nu == 2) { VUP(2, VT_Y_BIG) } else if (nu == 3) { VUP(3, VT_Y_BIG) } else { VUP(4, VT_Y_BIG) }
      } else {
        if (nu == 2) { VUP(2, VT_Y_SMALL) } else if (nu == 3) { VUP(3, VT_Y_SMALL) } else { VUP(4, VT_Y_SMALL) }
      }
#undef VUP
      std::swap(F.x, F.t);
      continue;
    }
    {
      const bool out = (l == 0 && nu == 1);
      if (out) k_v_post<Lv, R, true><<<nb, TPB, 0, st>>>(F, lv[l + 1], nd, F.t, om, z, dsc, sc);
      else k_v_post<Lv, R, false><<<nb, TPB, 0, st>>>(F, lv[l + 1], nd, F.t, om, nullptr, nullptr, sc);
      std::swap(F.x, F.t);
    }
    for (int k = 1; k < nu; ++k) {
      const bool last = (l == 0 && k == nu - 1);
      if (last) k_v_jacobi<Lv, R, true><<<nb, TPB, 0, st>>>(F, nd, F.x, F.t, om, z, dsc, sc);
      else k_v_jacobi<Lv, R, false><<<nb, TPB, 0, st>>>(F, nd, F.x, F.t, om, nullptr, nullptr, sc);
      std::swap(F.x, F.t);
    }
  }
}

// Sweeps per leg of hierarchy h: the option for momentum and pressure; at most
// 2 for transport, whose rows on reactive bands are not diagonally dominant
// (more damped-Jacobi sweeps amplify error modes there: measured 300-600
// iterations with 2, 1000-2300 with 4 on a Pe 47, Da 0.54 micromodel).
int sweeps(const vos_sim *s, int h) { return h == 3 ? std::min(2, s->opt.mg_nu) : s->nu_mom; }

// z = cycle(r) on hierarchy h, whose level 0 is the unscaled operator (the
// transport caller passes its row-scaled directions times the row diagonal).
template <typename R>
void smg_vcycle(vos_sim *s, int h, SLevel<R> *lv, const double *r, double *z, const double *sc, hipStream_t st,
                bool rg = false)
{
  vcycle<SLevel<R>, R>(s, lv, s->snlev[h], s->sainv[h], r, z, sc, 0.85, nullptr, 1.0, sweeps(s, h), st, rg);
}

// The V-cycle of aggregation hierarchy h runs its finest level's fused legs.
template <typename R>
bool smg_finest_fused(const vos_sim *s, int h, const SLevel<R> *lv)
{
  return coarse_start(s, lv, s->snlev[h]) > 0 && fused_level(s, lv[0], sweeps(s, h), nullptr);
}

// ---------------------------------------------------------------- stage S2

template <int D, typename R>
vos_status solve_momentum_t(vos_sim *s, const Lane &ln, SLevel<R> *lv, double dt, int *its, double *res, double *res0)
{
  const Dev &g = s->g;
  hipStream_t st = ln.st;
  double *part = ln.part;
  const unsigned n = g.nf[D];
  const int nb = grid_blocks(n);
  double *b = ln.vec[0], *r = ln.vec[1], *z = ln.vec[2], *pv = ln.vec[3], *q = ln.vec[4];
  double *x = s->ustar[D];
  double *sc = sc_block(s, SC_MOM + D);
  double *zero_flag = sc_block(s, SC_MISC) + S_COUNT;
  const double cvis = s->P.mu / (g.dx * g.dx);
  const double rt2 = s->opt.rtol_u * s->opt.rtol_u;
  // start: u^n, or with extrapolated starts the last predictor extrapolated
  // over the earlier ones
  const bool ex = s->opt.extrapolate && s->hist_u[D] >= 1;
  if (ex) {
    int h = s->hist_u[D] - 1;
    extrapolate(s, st, part, n, x, s->uprev[D], &h, D);
  }
  k_mom_rhs<D><<<nb, TPB, 0, st>>>(g, s->P, dt, s->eps, s->dmom[D], s->u[0], s->u[1], s->u[2], s->p, b, x, ex ? 0 : 1);
  if (hierarchy_due(s, H_MOM + D)) {
    k_smg_from_momentum<R, D><<<nb, TPB, 0, st>>>(g, cvis, s->dmom[D], lv[0]);
    smg_coarsen_all<R>(s, D, lv, st);
  }
  k_mom_apply<D><<<nb, TPB, 0, st>>>(g, cvis, s->dmom[D], x, q, part, zero_flag);
  k_cg_init<<<nb, TPB, 0, st>>>(n, b, q, s->dmom[D], r, z, pv, 0, part);
  k_cg_scal<<<1, TPB, 0, st>>>(0, part, nb, rt2, sc);
  smg_vcycle<R>(s, D, lv, r, z, sc, st);
  // the first direction is z (written here; unused when the start has converged)
  k_cg_zdots<<<nb, TPB, 0, st>>>(n, z, r, q, part, sc, pv);
  k_cg_scal<<<1, TPB, 0, st>>>(5, part, nb, rt2, sc);
  auto iter = [&]() {
    k_mom_apply<D><<<nb, TPB, 0, st>>>(g, cvis, s->dmom[D], pv, q, part, sc);
    k_cg_scal<<<1, TPB, 0, st>>>(1, part, nb, rt2, sc);
    k_cg_xr<<<nb, TPB, 0, st>>>(n, pv, q, s->dmom[D], x, r, z, 0, part, sc);
    k_cg_scal<<<1, TPB, 0, st>>>(3, part, nb, rt2, sc);
    smg_vcycle<R>(s, D, lv, r, z, sc, st);
    k_cg_zdots<<<nb, TPB, 0, st>>>(n, z, r, q, part, sc);
    k_cg_scal<<<1, TPB, 0, st>>>(4, part, nb, rt2, sc);
    k_cg_p<<<nb, TPB, 0, st>>>(n, z, pv, sc);
  };
  double res2, tol2;
  bool conv;
  vos_status stt = krylov_loop(s, ln, D, sc, s->opt.maxit_u, iter, its, &res2, &tol2, &conv);
  if (stt) return stt;
  k_mom_fix<D><<<nb, TPB, 0, st>>>(g, s->P.u_in, x);
  if (s->opt.extrapolate) s->hist_u[D] = conv ? std::min(NHIST + 1, s->hist_u[D] + 1) : 0;
  const double bn2 = ln.host[S_BN2];
  *res = bn2 > 0 ? std::sqrt(res2 / bn2) : 0.0;
  *res0 = bn2 > 0 ? std::sqrt(ln.host[S_RES0] / bn2) : 0.0;
  if (!conv) return fail(VOS_ERR_NOCONV, "momentum predictor did not converge");
  return VOS_OK;
}

template <int D>
vos_status solve_momentum(vos_sim *s, const Lane &ln, double dt, int *its, double *res, double *res0)
{
  if (s->opt.precision == VOS_MIXED) return solve_momentum_t<D, float>(s, ln, s->smgf[D], dt, its, res, res0);
  return solve_momentum_t<D, double>(s, ln, s->smgd[D], dt, its, res, res0);
}

// ---------------------------------------------------------------- stage S3

// Fluid-face transmissibility S dt / (rho dx): the global scale of the pressure hierarchy.
double pressure_scale(const vos_sim *s, double dt) { return s->g.S * dt / (s->P.rho * s->g.dx); }

template <typename R>
void mg_setup(vos_sim *s, MgLevel<R> *lv)
{
  hipStream_t st = s->stream;
  const Dev &g = s->g;
  const int nd = g.nd;
  const double inv_s = 1.0 / s->p_scale;
  k_mg_scaled_faces<R, 0><<<grid_blocks(g.nf[0]), TPB, 0, st>>>(g.nf[0], s->T[0], inv_s, lv[0]);
  k_mg_scaled_faces<R, 1><<<grid_blocks(g.nf[1]), TPB, 0, st>>>(g.nf[1], s->T[1], inv_s, lv[0]);
  if (nd == 3) k_mg_scaled_faces<R, 2><<<grid_blocks(g.nf[2]), TPB, 0, st>>>(g.nf[2], s->T[2], inv_s, lv[0]);
  k_mg_diag<R><<<grid_blocks(lv[0].nc), TPB, 0, st>>>(lv[0], nd);
  for (int l = 0; l + 1 < s->nlev; ++l) {
    k_mg_coarsen<R, 0><<<grid_blocks(lv[l + 1].nf[0]), TPB, 0, st>>>(lv[l], lv[l + 1], nd);
    k_mg_coarsen<R, 1><<<grid_blocks(lv[l + 1].nf[1]), TPB, 0, st>>>(lv[l], lv[l + 1], nd);
    if (nd == 3) k_mg_coarsen<R, 2><<<grid_blocks(lv[l + 1].nf[2]), TPB, 0, st>>>(lv[l], lv[l + 1], nd);
    k_mg_coarse_diag<R><<<grid_blocks(lv[l + 1].nc), TPB, 0, st>>>(lv[l], lv[l + 1], nd);
  }
  const MgLevel<R> &C = lv[s->nlev - 1];
  if (C.nc <= (unsigned)MG_COARSE_MAX) k_mg_coarse_inverse<R><<<1, GJ_TPB, 0, st>>>(C, nd, s->ainv);
}

template <typename R>
void mg_vcycle(vos_sim *s, MgLevel<R> *lv, const double *r, double *z, const double *sc)
{
  // A_R = A / p_scale, so z = A^-1 r is A_R^-1 (r / p_scale)
  vcycle<MgLevel<R>, R>(s, lv, s->nlev, s->ainv, r, z, sc, s->g.nd == 3 ? 6.0 / 7.0 : 0.8, nullptr,
                        1.0 / s->p_scale, s->opt.mg_nu, s->stream);
}

// ---------------------------------------------------------------- warm start


// Initial residual of p^n: r0 = b - A p^n (q = A p^n), kept in r0.  rd = r0 / sqrt(d)
// (the symmetrically scaled residual); partial sums of rd^2, r0^2 / d and b^2 / d.
__global__ void __launch_bounds__(TPB) k_ws_r0(unsigned n, const double *__restrict__ b, const double *__restrict__ q,
                                               const double *__restrict__ dg, double *__restrict__ r0,
                                               double *__restrict__ rd, double *__restrict__ part)
{
  double a = 0.0, r2 = 0.0, b2 = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double d = dg[i], r = b[i] - q[i];
    const double v = r / sqrt(d);
    r0[i] = r;
    rd[i] = v;
    a += v * v;
    r2 += r * r / d;
    b2 += b[i] * b[i] / d;
  }
  const double vv[3] = {a, r2, b2};
  write_partials<3>(vv, part);
}

// sc[0] = s0 = rms(rd), sc[1] = r0.D^-1.r0, sc[2] = b.D^-1.b.
__global__ void k_ws_stats(const double *__restrict__ part, int nb, unsigned n, double *__restrict__ sc)
{
  const double a = sum_partials(part, 0, nb);
  const double r2 = sum_partials(part, 1, nb);
  const double b2 = sum_partials(part, 2, nb);
  if (threadIdx.x == 0) {
    sc[0] = sqrt(a / (double)n);
    sc[1] = r2;
    sc[2] = b2;
  }
}

// Network input per cell: [eps_s, rd / s0, (i + 1/2) / nx, 1] (FP32, 4 channels),
// rd = r0 / sqrt(d).
__global__ void k_ws_input(Dev g, const double *__restrict__ eps, const double *__restrict__ rd,
                           const double *__restrict__ sc, float *__restrict__ x)
{
  const double s0 = sc[0];
  const double inv = s0 > 0.0 ? 1.0 / s0 : 0.0;
  for (unsigned id = xbeg(g.nc); id < xend(g.nc); id += xstride()) {
    const unsigned i = id % (unsigned)g.n[0];
    float4 v;
    v.x = (float)(1.0 - eps[id]);
    v.y = (float)(rd[id] * inv);
    v.z = (float)((i + 0.5) / g.n[0]);
    v.w = 1.0f;
    reinterpret_cast<float4 *>(x)[id] = v;
  }
}

// Search direction from the network output, back from the scaled space:
// v = y / sqrt(d) (FP64) where the cell carries flow (eps > 2 eps_min), 0 in
// intact solid: there d ~ 1e-30 would turn output noise into huge pressure
// changes that the flow does not see but the Jacobi-scaled residual does.
__global__ void k_ws_dir(unsigned n, const float *__restrict__ y, const double *__restrict__ dg,
                         const double *__restrict__ eps, double eps_live, double *__restrict__ v)
{
  for (unsigned i = xbeg(n); i < xend(n); i += xstride())
    v[i] = eps[i] > eps_live ? (double)y[i] / sqrt(dg[i]) : 0.0;
}

// Partial sums of v.r0, v.(A v), (A v).D^-1.r0 and (A v).D^-1.(A v) (q = A v).
__global__ void __launch_bounds__(TPB) k_ws_dots(unsigned n, const double *__restrict__ v,
                                                 const double *__restrict__ r0, const double *__restrict__ q,
                                                 const double *__restrict__ dg, double *__restrict__ part)
{
  double a = 0.0, c = 0.0, e = 0.0, f = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    a += v[i] * r0[i];
    c += v[i] * q[i];
    e += q[i] * r0[i] / dg[i];
    f += q[i] * q[i] / dg[i];
  }
  const double vv[4] = {a, c, e, f};
  write_partials<4>(vv, part);
}

// Step along v minimising the Jacobi-scaled residual of p^n + alpha v (the
// norm the solve's stopping rule measures): alpha = (Av).D^-1.r0 /
// (Av).D^-1.(Av), 0 if that is not defined.  sc[4] = alpha, sc[5] = the
// decrease of the squared A-norm error this step gives, 2 alpha v.r0 -
// alpha^2 v.Av (may be negative).
__global__ void k_ws_alpha(const double *__restrict__ part, int nb, double *__restrict__ sc)
{
  const double a = sum_partials(part, 0, nb);
  const double c = sum_partials(part, 1, nb);
  const double e = sum_partials(part, 2, nb);
  const double f = sum_partials(part, 3, nb);
  if (threadIdx.x == 0) {
    const bool ok = f > 0.0 && isfinite(e / f);
    const double al = ok ? e / f : 0.0;
    sc[4] = al;
    sc[5] = 2.0 * al * a - al * al * c;
  }
}

// p = p^n + alpha v.
__global__ void k_ws_guess(unsigned n, const double *__restrict__ pn, const double *__restrict__ v,
                           const double *__restrict__ sc, double *__restrict__ p)
{
  const double al = sc[4];
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) p[i] = pn[i] + al * v[i];
}

// v = p - pn.
__global__ void k_ws_diff(unsigned n, const double *__restrict__ p, const double *__restrict__ pn, double *__restrict__ v)
{
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) v[i] = p[i] - pn[i];
}

// Partial sums of (b - q)^2 / d.
__global__ void __launch_bounds__(TPB) k_ws_res(unsigned n, const double *__restrict__ b, const double *__restrict__ q,
                                                const double *__restrict__ dg, double *__restrict__ part)
{
  double a = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double r = b[i] - q[i];
    a += r * r / dg[i];
  }
  const double vv[1] = {a};
  write_partials<1>(vv, part);
}

__global__ void k_ws_store(const double *__restrict__ part, int nb, double *__restrict__ out)
{
  const double a = sum_partials(part, 0, nb);
  if (threadIdx.x == 0) out[0] = a;
}

// Training target sqrt(d) (p - p^n) / (gain s0) as FP32 (0 where s0 = 0): the
// increment in the symmetrically scaled space, whose squared norm weights each
// cell by its diagonal as the A-norm does.
__global__ void k_ws_target(unsigned n, const double *__restrict__ p, const double *__restrict__ pn,
                            const double *__restrict__ dg, double scale, float *__restrict__ t)
{
  const double inv = scale > 0.0 ? 1.0 / scale : 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) t[i] = (float)(sqrt(dg[i]) * (p[i] - pn[i]) * inv);
}

// Build the network input from the solve's initial residual.  With the guess
// enabled, take the network output as a search direction v from p^n with the
// step alpha that minimises the Jacobi-scaled residual (the stopping rule's
// norm), and start from p^n + alpha v if that residual is smaller than p^n's.
// s->p holds p^n on entry, the start on exit.  Scratch: q, rd, r0 (CG
// overwrites them).
vos_status warm_start(vos_sim *s, const double *b, double *q, double *rd, double *r0, const double *zero_flag)
{
  const Dev &g = s->g;
  hipStream_t st = s->stream;
  const unsigned n = g.nc;
  const int nb = grid_blocks(n);
  double *sc = sc_block(s, SC_WS);
  float *x = vosint::unet_input(s->net);
  p_apply(s, s->pn, q, zero_flag);
  k_ws_r0<<<nb, TPB, 0, st>>>(n, b, q, s->pdiag, r0, rd, s->part);
  k_ws_stats<<<1, TPB, 0, st>>>(s->part, nb, n, sc);
  k_ws_input<<<nb, TPB, 0, st>>>(g, s->eps, rd, sc, x);
  s->ws_used = 0;
  s->ws_res_guess = 0.0;
  if (s->ws_use) {
    if (vos_status e = vosint::unet_forward_on(s->net, st)) return e;
    double *v = rd;   // the scaled residual is no longer needed
    k_ws_dir<<<nb, TPB, 0, st>>>(n, vosint::unet_output(s->net), s->pdiag, s->eps, 2.0 * s->P.eps_min, v);
    p_apply(s, v, q, zero_flag);
    k_ws_dots<<<nb, TPB, 0, st>>>(n, v, r0, q, s->pdiag, s->part);
    k_ws_alpha<<<1, TPB, 0, st>>>(s->part, nb, sc);
    k_ws_guess<<<nb, TPB, 0, st>>>(n, s->pn, v, sc, s->p);
    p_apply(s, s->p, q, zero_flag);
    k_ws_res<<<nb, TPB, 0, st>>>(n, b, q, s->pdiag, s->part);
    k_ws_store<<<1, TPB, 0, st>>>(s->part, nb, sc + 3);
  }
  HIP_TRY(hipGetLastError());
  if (vos_status e = read_back(s, sc, 6)) return e;
  const double *h = s->host;
  s->ws_s0 = h[0];
  s->ws_sampled = true;
  const double bn = h[2] > 0.0 ? h[2] : 1.0;
  s->ws_res_prev = std::sqrt(h[1] / bn);
  if (s->ws_use) {
    s->ws_res_guess = std::sqrt(h[3] / bn);
    s->ws_drop = h[5];
    if (h[3] < h[1] && std::isfinite(h[3])) {
      s->ws_used = 1;
    } else {
      HIP_TRY(hipMemcpyAsync(s->p, s->pn, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    }
  }
  return VOS_OK;
}

// Sum of the continuity source's partials into slot 16 of the diag block.
__global__ void k_src_sum(const double *__restrict__ part, int nb, double *__restrict__ out)
{
  const double v = sum_partials(part, 0, nb);
  if (threadIdx.x == 0) out[0] = v;
}

template <typename R>
vos_status solve_pressure_t(vos_sim *s, MgLevel<R> *lv, int gid, int h, int *its, double *res, double *res0,
                            const double *guess)
{
  const Dev &g = s->g;
  hipStream_t st = s->stream;
  const unsigned n = g.nc;
  const int nb = grid_blocks(n);
  double *b = s->vec[0], *r = s->vec[1], *z = s->vec[2], *pv = s->vec[3], *q = s->vec[4];
  double *sc = sc_block(s, SC_P);
  double *zero_flag = sc_block(s, SC_MISC) + S_COUNT;
  const double rt2 = s->opt.rtol_p * s->opt.rtol_p;
  if (hierarchy_due(s, h)) mg_setup<R>(s, lv);
  HIP_TRY(hipMemcpyAsync(s->pn, s->p, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (guess) {   // a caller's start (vos_solve_pressure); the right-hand side keeps p^n (pn)
    HIP_TRY(hipMemcpyAsync(s->p, guess, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  } else if (s->opt.extrapolate && !s->net) {   // the start only; the right-hand side keeps p^n (pn)
    extrapolate(s, st, s->part, n, s->p, s->pprev, &s->hist_p, 3);
  }
  const bool src = s->P.transient != 0;
  k_p_rhs<<<nb, TPB, 0, st>>>(g, s->T[0], s->T[1], s->T[2], s->pn, s->ustar[0], s->ustar[1], s->ustar[2], b,
                              src ? s->rbar : nullptr, s->P.Vm - s->P.Vm_f, s->part);
  if (src) k_src_sum<<<1, TPB, 0, st>>>(s->part, nb, sc_block(s, SC_DIAG) + 16);
  if (s->net)
    if (vos_status e = warm_start(s, b, q, z, pv, zero_flag)) return e;
  p_apply(s, s->p, q, zero_flag);
  k_cg_init<<<nb, TPB, 0, st>>>(n, b, q, s->pdiag, r, z, pv, 0, s->part);
  k_cg_scal<<<1, TPB, 0, st>>>(0, s->part, nb, rt2, sc);
  mg_vcycle<R>(s, lv, r, z, sc);
  // the first direction is z (written here; unused when the start has converged)
  k_cg_zdots<<<nb, TPB, 0, st>>>(n, z, r, q, s->part, sc, pv);
  k_cg_scal<<<1, TPB, 0, st>>>(5, s->part, nb, rt2, sc);
  auto iter = [&]() {
    const int nbq = p_apply(s, pv, q, sc);
    k_cg_scal<<<1, TPB, 0, st>>>(1, s->part, nbq, rt2, sc);
    k_cg_xr<<<nb, TPB, 0, st>>>(n, pv, q, s->pdiag, s->p, r, z, 0, s->part, sc);
    k_cg_scal<<<1, TPB, 0, st>>>(3, s->part, nb, rt2, sc);
    mg_vcycle<R>(s, lv, r, z, sc);
    k_cg_zdots<<<nb, TPB, 0, st>>>(n, z, r, q, s->part, sc);
    k_cg_scal<<<1, TPB, 0, st>>>(4, s->part, nb, rt2, sc);
    k_cg_p<<<nb, TPB, 0, st>>>(n, z, pv, sc);
  };
  double res2, tol2;
  bool conv;
  Stall stall;
  const bool mixed = std::is_same<R, float>::value;
  if (mixed) {
    stall.window = P_STALL_WINDOW;
    stall.cap = s->opt.p_fp32_its;
  }
  s->it_p_fp64 = 0;
  vos_status stt = krylov_loop(s, main_lane(s), gid, sc, s->opt.maxit_p, iter, its, &res2, &tol2, &conv, mixed ? &stall : nullptr);
  if (stt) return stt;
  s->p_res0 = s->host[S_BN2] > 0 ? std::sqrt(s->host[S_RES0] / s->host[S_BN2]) : 0.0;
  if (!mixed && s->opt.precision == VOS_MIXED) s->it_p_fp64 = *its;   // a solve after an FP32 stall
  if (stall.hit && !conv) {
    if (!stall.by_cap) s->p_fp64_sticky = true;   // later solves of this geometry start in FP64
    // continue the same flexible CG with an FP64 hierarchy built over the FP32 one's memory
    // (the next solve rebuilds the FP32 hierarchy)
    mg_setup<double>(s, s->mgd);
    s->mg_age[H_P64] = 1;
    s->mg_age[H_P] = 1 << 30;
    auto iter64 = [&]() {
      const int nbq = p_apply(s, pv, q, sc);
      k_cg_scal<<<1, TPB, 0, st>>>(1, s->part, nbq, rt2, sc);
      k_cg_xr<<<nb, TPB, 0, st>>>(n, pv, q, s->pdiag, s->p, r, z, 0, s->part, sc);
      k_cg_scal<<<1, TPB, 0, st>>>(3, s->part, nb, rt2, sc);
      mg_vcycle<double>(s, s->mgd, r, z, sc);
      k_cg_zdots<<<nb, TPB, 0, st>>>(n, z, r, q, s->part, sc);
      k_cg_scal<<<1, TPB, 0, st>>>(4, s->part, nb, rt2, sc);
      k_cg_p<<<nb, TPB, 0, st>>>(n, z, pv, sc);
    };
    const int its32 = *its;
    stt = krylov_loop(s, main_lane(s), 5, sc, std::max(1, s->opt.maxit_p - its32), iter64, its, &res2, &tol2, &conv);
    if (stt) return stt;
    s->it_p_fp64 = *its - its32;
  }
  s->ws_frac = 0.0;
  if (s->net && s->ws_use) {
    // squared A-norm of the increment dp = p^{n+1} - p^n: the initial error of a start at p^n
    k_ws_diff<<<nb, TPB, 0, st>>>(n, s->p, s->pn, z);
    const int nbq = p_apply(s, z, q, zero_flag);
    k_ws_store<<<1, TPB, 0, st>>>(s->part, nbq, sc_block(s, SC_WS) + 6);
    HIP_TRY(hipGetLastError());
    if (vos_status e = read_back(s, sc_block(s, SC_WS) + 6, 1)) return e;
    const double e2 = s->host[0];
    s->ws_frac = (e2 > 0.0 && s->ws_used) ? std::min(1.0, s->ws_drop / e2) : 0.0;
  }
  const double bn2 = s->host[S_BN2];
  *res = bn2 > 0 ? std::sqrt(res2 / bn2) : 0.0;
  *res0 = s->p_res0;
  if (!conv) return fail(VOS_ERR_NOCONV, "pressure solve did not converge");
  return VOS_OK;
}

vos_status solve_pressure(vos_sim *s, int *its, double *res, double *res0, const double *guess = nullptr)
{
  // mixed precision: the FP32 hierarchy until one of its solves stalls on this geometry, then
  // FP64 (its iteration chunk captured under its own graph slot)
  if (s->opt.precision == VOS_MIXED && !s->p_fp64_sticky)
    return solve_pressure_t<float>(s, s->mgf, 3, H_P, its, res, res0, guess);
  const bool mixed = s->opt.precision == VOS_MIXED;
  return solve_pressure_t<double>(s, s->mgd, mixed ? 5 : 3, mixed ? H_P64 : H_P, its, res, res0, guess);
}

// ---------------------------------------------------------------- stage S4

void launch_correct(vos_sim *s)
{
  const Dev &g = s->g;
  hipStream_t st = s->stream;
  k_correct<0><<<grid_blocks(g.nf[0]), TPB, 0, st>>>(g, s->ustar[0], s->af[0], s->p, s->pn, s->u[0]);
  k_correct<1><<<grid_blocks(g.nf[1]), TPB, 0, st>>>(g, s->ustar[1], s->af[1], s->p, s->pn, s->u[1]);
  if (g.nd == 3) k_correct<2><<<grid_blocks(g.nf[2]), TPB, 0, st>>>(g, s->ustar[2], s->af[2], s->p, s->pn, s->u[2]);
}

// ---------------------------------------------------------------- stage S5

template <typename R>
vos_status solve_transport_t(vos_sim *s, SLevel<R> *lv, double dt, int vl, int *its, double *res, double *res0)
{
  const Dev &g = s->g;
  hipStream_t st = s->stream;
  const unsigned n = g.nc;
  const int nb = grid_blocks(n);
  // the shadow residual rh is a hash of the cell index, formed where it is read
  double *b = s->vec[0], *r = s->vec[1], *pv = s->vec[3], *v = s->vec[4], *sv = s->vec[5], *t = s->vec[6],
         *y = s->vec[7], *ph = s->vec[8], *sh = s->vec[9];
  double *sc = sc_block(s, SC_C);
  double *zero_flag = sc_block(s, SC_MISC) + S_COUNT;
  const int H = 3;
  const double rt2 = s->opt.rtol_c * s->opt.rtol_c;
  HIP_TRY(hipMemcpyAsync(s->cold, s->c, n * sizeof(double), hipMemcpyDeviceToDevice, st));
  if (s->opt.extrapolate) {   // the start only; the deferred correction keeps c^n (cold)
    extrapolate(s, st, s->part, n, s->c, s->cprev, &s->hist_c, 4);
  }
  auto assemble = [&]() {
    k_adr_assemble<<<nb, TPB, 0, st>>>(g, s->P, s->eps, s->u[0], s->u[1], s->u[2], s->w[0], s->w[1], s->w[2],
                                       s->cold, s->gmag, sc_block(s, SC_MISC), s->off, b, s->tdiag, s->tdif, vl, dt,
                                       s->eps_prev, s->c0);
  };
  assemble();
  // rebuilt every step: a transport hierarchy one step old can stall BiCGStab on
  // strongly reactive instances (Da ~ 1), where the rows change most between steps
  k_smg_from_transport<R><<<nb, TPB, 0, st>>>(n, g.nd, s->off, s->tdiag, s->tdif, lv[0]);
  smg_coarsen_all<R>(s, H, lv, st);
  k_adr_apply<1><<<nb, TPB, 0, st>>>(g, s->off, s->c, y, s->c, s->part, zero_flag);
  k_bi_init<<<nb, TPB, 0, st>>>(n, b, y, r, nullptr, pv, v, s->part);
  k_bi_scal<<<1, TPB, 0, st>>>(0, s->part, nb, rt2, sc);
  // the directions times the row diagonal, the input of the cycle built on the
  // unscaled rows (y is free after the start; b stays for the true residual);
  // where the cycle's finest level runs the fused legs they form it from the
  // directions and the level's diagonal (= the row diagonal) themselves
  const bool rg = smg_finest_fused(s, H, lv);
  double *pd = rg ? nullptr : s->vec[10], *sd = rg ? nullptr : y;
  auto iter = [&]() {
    k_bi_p<<<nb, TPB, 0, st>>>(n, r, v, pv, pd, s->tdiag, sc);
    smg_vcycle<R>(s, H, lv, rg ? pv : pd, ph, sc, st, rg);
    k_adr_apply<1, true><<<nb, TPB, 0, st>>>(g, s->off, ph, v, nullptr, s->part, sc);
    k_bi_scal<<<1, TPB, 0, st>>>(1, s->part, nb, rt2, sc);
    k_bi_s<<<nb, TPB, 0, st>>>(n, r, v, sv, sd, s->tdiag, s->part, sc);
    k_bi_scal<<<1, TPB, 0, st>>>(2, s->part, nb, rt2, sc);
    smg_vcycle<R>(s, H, lv, rg ? sv : sd, sh, sc, st, rg);
    k_adr_apply<2><<<nb, TPB, 0, st>>>(g, s->off, sh, t, sv, s->part, sc);
    k_bi_scal<<<1, TPB, 0, st>>>(3, s->part, nb, rt2, sc);
    k_bi_xr<<<nb, TPB, 0, st>>>(n, ph, sh, sv, t, s->c, r, s->part, sc);
    k_bi_scal<<<1, TPB, 0, st>>>(4, s->part, nb, rt2, sc);
  };
  double res2, tol2;
  bool conv;
  vos_status stt = krylov_loop(s, main_lane(s), 4, sc, s->opt.maxit_c, iter, its, &res2, &tol2, &conv);
  if (stt) return stt;
  double bn2 = s->host[S_BN2];
  *res0 = bn2 > 0 ? std::sqrt(s->host[S_RES0] / bn2) : 0.0;
  // BiCGStab's recurrence residual drifts from b - A c; accept convergence only
  // once the true residual meets the tolerance, else restart from the iterate
  for (int restart = 0; conv && restart < 4; ++restart) {
    k_adr_apply<1><<<nb, TPB, 0, st>>>(g, s->off, s->c, y, s->c, s->part, zero_flag);
    k_bi_true_res<<<nb, TPB, 0, st>>>(n, b, y, s->part);
    k_bi_true_scal<<<1, TPB, 0, st>>>(s->part, nb, sc);
    HIP_TRY(hipGetLastError());
    if (vos_status e = read_back(s, sc, S_COUNT)) return e;
    if (s->host[S_TRUE] <= s->host[S_TOL2]) { res2 = s->host[S_TRUE]; break; }
    int more = 0;
    k_bi_init<<<nb, TPB, 0, st>>>(n, b, y, r, nullptr, pv, v, s->part);
    k_bi_scal<<<1, TPB, 0, st>>>(0, s->part, nb, rt2, sc);
    stt = krylov_loop(s, main_lane(s), 4, sc, std::max(1, s->opt.maxit_c - *its), iter, &more, &res2, &tol2, &conv);
    if (stt) return stt;
    *its += more;
  }
  bn2 = s->host[S_BN2];
  *res = bn2 > 0 ? std::sqrt(res2 / bn2) : 0.0;
  if (!conv) return fail(VOS_ERR_NOCONV, "transport solve did not converge");
  return VOS_OK;
}

vos_status solve_transport(vos_sim *s, double dt, int *its, double *res, double *res0, int vl = 1)
{
  return solve_transport_t<double>(s, s->smgd[3], dt, vl, its, res, res0);   // FP64 hierarchy in both precisions
}

// ---------------------------------------------------------------- stages S6-S7

// Sum the reaction / update partials into the diag scalar block:
// [0] sink sum, [1] rate sum, [2..13] k_eps_update slots 0..11, [14] max |d eps|
// ([15]: the shortened solid step, written by k_solid_dt; [16]: the continuity
// source sum, written by k_src_sum).
__global__ void k_diag_final(const double *__restrict__ prt, const double *__restrict__ pupd,
                             const double *__restrict__ pmax, int nb, double *__restrict__ out)
{
  double v[15];
  v[0] = sum_partials(prt, 0, nb);
  v[1] = sum_partials(prt, 1, nb);
  for (int q = 0; q < 12; ++q) v[2 + q] = sum_partials(pupd, q, nb);
  v[14] = max_partials(pmax, 0, nb);
  if (threadIdx.x == 0)
    for (int q = 0; q < 15; ++q) out[q] = v[q];
}

// p = pn + relax (p - pn): SIMPLE's explicit pressure under-relaxation.
__global__ void k_relax(unsigned n, double relax, const double *__restrict__ pn, double *__restrict__ p)
{
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) p[i] = pn[i] + relax * (p[i] - pn[i]);
}

// Partials of sum (a - b)^2 and sum a^2 over n entries (slots 0 and 1 of part).
__global__ void __launch_bounds__(TPB) k_du(unsigned n, const double *__restrict__ a, const double *__restrict__ b,
                                            double *__restrict__ part)
{
  double d2 = 0.0, a2 = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double d = a[i] - b[i];
    d2 += d * d;
    a2 += a[i] * a[i];
  }
  const double v[2] = {d2, a2};
  write_partials<2>(v, part);
}

// out[0] = sqrt(sum (u - u_prev)^2 / sum u^2) over the face grids whose partials
// k_du left at slots 0-1, 2-3 and 4-5 (nb2 = 0: no third grid).
__global__ void k_du_final(const double *__restrict__ part, int nb0, int nb1, int nb2, double *__restrict__ out)
{
  double d2 = sum_partials(part, 0, nb0) + sum_partials(part, 2, nb1);
  double a2 = sum_partials(part, 1, nb0) + sum_partials(part, 3, nb1);
  if (nb2 > 0) {
    d2 += sum_partials(part, 4, nb2);
    a2 += sum_partials(part, 5, nb2);
  }
  if (threadIdx.x == 0) out[0] = a2 > 0.0 ? sqrt(d2 / a2) : 0.0;
}

// Partials of the rates: 2 slots after the update's 12.
double *rate_partials(vos_sim *s) { return s->part + 12 * MAXB; }

// Reaction rates Rbar from the current c (S6); the per-block maxima of the
// rates that may set the solid step go to part_max.
void launch_rates(vos_sim *s)
{
  const Dev &g = s->g;
  k_react<<<grid_blocks(g.nc), TPB, 0, s->stream>>>(g, s->P, s->eps, s->c, s->cold, s->w[0], s->w[1], s->w[2],
                                                     s->gmag, sc_block(s, SC_MISC), s->rbar, rate_partials(s),
                                                     s->part_max, s->opt.deps_max);
}

double solid_nominal(const vos_sim *s, double dt) { return s->opt.solid_dt > 0.0 ? s->opt.solid_dt : dt; }

// Solid update (S7) from the rates of launch_rates, and the diagnostic sums.
void launch_update(vos_sim *s, double dt, int freeze)
{
  const Dev &g = s->g;
  hipStream_t st = s->stream;
  const int nb = grid_blocks(g.nc);
  // the solid step (slot 15 of the diag block) when it may be shortened;
  // k_eps_update reuses part_max after k_solid_dt has read it
  double *dts = nullptr;
  s->solid_dt_dev = s->opt.deps_max > 0.0 && !freeze;
  if (s->solid_dt_dev) {
    dts = sc_block(s, SC_DIAG) + 15;
    k_solid_dt<<<1, TPB, 0, st>>>(s->part_max, nb, dt, s->opt.deps_max, dts);
  }
  k_eps_update<<<nb, TPB, 0, st>>>(g, s->P, dt, dts, freeze, s->eps, s->rbar, s->c, s->p, s->u[0], s->gmag,
                                   s->part, s->part_max, s->eps_prev, s->c0);
  k_diag_final<<<1, TPB, 0, st>>>(rate_partials(s), s->part, s->part_max, nb, sc_block(s, SC_DIAG));
}

vos_status fill_diag(vos_sim *s, double dt, vos_diag *dg)
{
  // one synchronisation: lambda (misc block) to host[0], the 17 sums to host[2..18]
  HIP_TRY(hipMemcpyAsync(s->host, sc_block(s, SC_MISC), 2 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipMemcpyAsync(s->host + 2, sc_block(s, SC_DIAG), 17 * sizeof(double), hipMemcpyDeviceToHost, s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  const double lam = s->host[0];
  const double *h = s->host + 2;
  const Dev &g = s->g;
  const double V = g.V;
  const double sink = h[0], rate = h[1];
  dg->lambda = lam;
  dg->clipped_volume = h[2];
  const double dvol = h[3];
  dg->solid_volume = h[4];
  dg->porosity = h[5] / (double)g.nc;
  dg->acid_in = h[6];
  dg->acid_out = h[7];
  const double nin = (double)g.n[1] * g.n[2];
  dg->U_D = h[12] / (nin * g.S);
  if (g.drive) {
    dg->dP = s->P.p_in - s->P.p_out;
    dg->K = dg->dP != 0.0 ? s->P.mu * dg->U_D * g.n[0] * g.dx / dg->dP : 0.0;
  } else {
    dg->dP = h[8] / nin - s->P.p_out;
    dg->K = dg->dP != 0.0 ? s->P.mu * s->P.u_in * (g.n[0] - 0.5) * g.dx / dg->dP : 0.0;
  }
  const double cg = h[9], ec = h[10], area = h[11];
  dg->surface_area = area;
  const double a = area / (g.nc * V);
  dg->alpha = (a > 0.0 && ec > 0.0) ? cg / (a * ec) : 0.0;
  dg->acid_accum = s->P.transient ? h[13] : 0.0;
  dg->max_deps = h[14];
  dg->acid_consumed = s->P.zeta * sink;
  dg->solid_rate = rate;
  dg->acid_balance_rel =
      dg->acid_in != 0.0 ? (dg->acid_in - dg->acid_out - dg->acid_consumed - dg->acid_accum) / dg->acid_in : 0.0;
  dg->dt_solid = s->solid_dt_dev ? h[15] : dt;
  dg->div_source = s->P.transient ? h[16] : 0.0;
  const double dts = dg->dt_solid;
  const double ref = dts * s->P.Vm * std::fabs(rate);
  dg->solid_balance_rel = ref > 0.0 ? (dvol - dts * s->P.Vm * rate + dg->clipped_volume) / ref : 0.0;
  dg->R_omega = s->P.Vm > 0.0 ? dvol / ((double)g.nc * V) / (s->P.Vm * dts) : 0.0;
  return VOS_OK;
}

// The momentum predictor of every component (S2): each component on its own
// momentum lane, components 1 and 2 driven from further host threads; returns
// the largest initial relative residual of the solves in *r0.
vos_status momentum_stage(vos_sim *s, double dt, vos_diag *dg, double *r0, vos_status *rc)
{
  hipStream_t st = s->stream;
  const int nl = s->g.nd == 3 ? 3 : 2;
  HIP_TRY(hipEventRecord(s->fork, st));
  for (int k = 0; k < nl; ++k) HIP_TRY(hipStreamWaitEvent(s->lane_stream[k], s->fork, 0));
  vos_status r1 = VOS_OK, r3 = VOS_OK;
  std::string m1, m3;
  double q[3] = {0.0, 0.0, 0.0};
  std::thread t1([&]() {
    r1 = solve_momentum<1>(s, momentum_lane(s, 1), dt, &dg->it_u[1], &dg->res_u[1], &q[1]);
    if (r1) m1 = vos_last_error();
  });
  std::thread t2;
  if (nl == 3)
    t2 = std::thread([&]() {
      r3 = solve_momentum<2>(s, momentum_lane(s, 2), dt, &dg->it_u[2], &dg->res_u[2], &q[2]);
      if (r3) m3 = vos_last_error();
    });
  vos_status r0s = solve_momentum<0>(s, momentum_lane(s, 0), dt, &dg->it_u[0], &dg->res_u[0], &q[0]);
  std::string m0 = r0s ? std::string(vos_last_error()) : std::string();
  t1.join();
  if (t2.joinable()) t2.join();
  for (int k = 0; k < nl; ++k) {
    HIP_TRY(hipEventRecord(s->join[k], s->lane_stream[k]));
    HIP_TRY(hipStreamWaitEvent(st, s->join[k], 0));
  }
  *r0 = std::max(q[0], std::max(q[1], q[2]));
  // component order for the reported status: 0, 1, 2 (device errors end the step)
  const vos_status rr[3] = {r0s, r1, r3};
  const std::string *mm[3] = {&m0, &m1, &m3};
  for (int k = 0; k < 3; ++k)
    if (rr[k] == VOS_ERR_DEVICE) return fail(rr[k], *mm[k]);
  for (int k = 0; k < 3; ++k)
    if (rr[k] && !*rc) *rc = fail(rr[k], *mm[k]);
  return VOS_OK;
}

// New time-step size: the captured V-cycles and the pressure hierarchy hold
// 1/p_scale, which depends on it.
void set_time_step(vos_sim *s, double dt)
{
  // every matrix carries dt (the momentum diagonal rho eps / dt, the pressure
  // transmissibilities through it): a new dt rebuilds every hierarchy at its next solve
  const double ps = pressure_scale(s, dt);
  if (ps != s->p_scale) {
    drop_graphs(s);
    s->p_scale = ps;
    hierarchies_stale(s);
  }
}

vos_status one_step(vos_sim *s, double dt, int flags, vos_diag *dg)
{
  hipStream_t st = s->stream;
  std::memset(dg, 0, sizeof(*dg));
  vos_status rc = VOS_OK, r2;
  set_time_step(s, dt);
  HIP_TRY(hipEventRecord(s->ev[0], st));
  if (s->P.transient)   // c at the step's start, for the storage term
    HIP_TRY(hipMemcpyAsync(s->c0, s->c, s->g.nc * sizeof(double), hipMemcpyDeviceToDevice, st));
  launch_coefficients(s, dt);
  float ms = 0.f;
  // one pass, or the SIMPLE loop (Appendix B) with eps frozen until every
  // solve starts within outer_tol of its solution
  const int nout = s->opt.simple ? s->opt.outer_max : 1;
  for (int it = 0; it < nout; ++it) {
    double q = 0.0, worst = 0.0;
    HIP_TRY(hipEventRecord(s->ev[1], st));
    if (vos_status e = momentum_stage(s, dt, dg, &q, &rc)) return e;
    worst = std::max(worst, q);
    HIP_TRY(hipEventRecord(s->ev[2], st));
    r2 = solve_pressure(s, &dg->it_p, &dg->res_p, &q);
    if (r2 == VOS_ERR_DEVICE) return r2;
    if (r2 && !rc) rc = r2;
    worst = std::max(worst, q);
    dg->guess = s->net ? s->ws_used : -1;
    dg->res0_prev = s->net ? s->ws_res_prev : 0.0;
    dg->res0_guess = s->net ? s->ws_res_guess : 0.0;
    dg->guess_error_drop = s->net ? s->ws_frac : 0.0;
    dg->it_p_fp64 = s->it_p_fp64;
    HIP_TRY(hipEventRecord(s->ev[3], st));
    launch_correct(s);
    if (s->opt.simple) k_relax<<<grid_blocks(s->g.nc), TPB, 0, st>>>(s->g.nc, s->opt.relax_p, s->pn, s->p);
    HIP_TRY(hipEventRecord(s->ev[4], st));
    r2 = solve_transport(s, dt, &dg->it_c, &dg->res_c, &q);
    if (r2 == VOS_ERR_DEVICE) return r2;
    if (r2 && !rc) rc = r2;
    worst = std::max(worst, q);
    HIP_TRY(hipEventRecord(s->ev[5], st));
    launch_rates(s);
    HIP_TRY(hipEventRecord(s->ev[6], st));
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipEventSynchronize(s->ev[6]));
    if (it == 0) {   // coefficients: from the step's start to the first momentum stage
      HIP_TRY(hipEventElapsedTime(&ms, s->ev[0], s->ev[1]));
      dg->t_ms[0] = ms;
    }
    for (int k = 1; k < 6; ++k) {
      HIP_TRY(hipEventElapsedTime(&ms, s->ev[k], s->ev[k + 1]));
      dg->t_ms[k] += ms;
    }
    dg->outer_its = it + 1;
    dg->outer_res = worst;
    if (rc) break;
    if (s->opt.simple && worst <= s->opt.outer_tol) break;
  }
  HIP_TRY(hipEventRecord(s->ev[5], st));
  launch_update(s, solid_nominal(s, dt), flags & VOS_FREEZE_SOLID);
  HIP_TRY(hipEventRecord(s->ev[6], st));
  HIP_TRY(hipGetLastError());
  r2 = fill_diag(s, solid_nominal(s, dt), dg);
  if (r2) return r2;
  HIP_TRY(hipEventElapsedTime(&ms, s->ev[5], s->ev[6]));
  dg->t_ms[5] += ms;
  if (rc) {
    std::string m = g_err;
    return fail(rc, m);
  }
  return VOS_OK;
}

double *field_ptr(vos_sim *s, int field, size_t *n, bool *writable)
{
  const Dev &g = s->g;
  *writable = true;
  switch (field) {
    case VOS_FIELD_EPS: *n = g.nc; return s->eps;
    case VOS_FIELD_UX: *n = g.nf[0]; return s->u[0];
    case VOS_FIELD_UY: *n = g.nf[1]; return s->u[1];
    case VOS_FIELD_UZ: *n = g.nf[2]; return s->u[2];
    case VOS_FIELD_P: *n = g.nc; return s->p;
    case VOS_FIELD_C: *n = g.nc; return s->c;
    case VOS_FIELD_USTAR_X: *writable = false; *n = g.nf[0]; return s->ustar[0];
    case VOS_FIELD_USTAR_Y: *writable = false; *n = g.nf[1]; return s->ustar[1];
    case VOS_FIELD_USTAR_Z: *writable = false; *n = g.nf[2]; return s->ustar[2];
    case VOS_FIELD_RBAR: *writable = false; *n = g.nc; return s->rbar;
    case VOS_FIELD_GMAG: *writable = false; *n = g.nc; return s->gmag;
    case VOS_FIELD_PDIAG: *writable = false; *n = g.nc; return s->pdiag;
    default: return nullptr;
  }
}

__global__ void k_set_eps(unsigned n, const double *__restrict__ es, double eps_min, double *__restrict__ eps,
                          int *__restrict__ bad)
{
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double v = es[i];
    if (!(v >= 0.0 && v <= 1.0)) bad[0] = 1;
    double e = 1.0 - v;
    e = e < eps_min ? eps_min : (e > 1.0 ? 1.0 : e);
    eps[i] = e;
  }
}

__global__ void k_fill(unsigned n, double v, double *__restrict__ a)
{
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) a[i] = v;
}

// Velocity the inlet faces start from: u_in under the velocity drive, rest
// (0) under the pressure drive, where they are unknowns.
double inlet_velocity(const vos_sim *s) { return s->g.drive ? 0.0 : s->P.u_in; }

// Inlet faces (i = 0) of the x grid get u_in.
__global__ void k_inlet(Dev g, double u_in, double *__restrict__ ux)
{
  const unsigned n = (unsigned)g.n[1] * g.n[2];
  for (unsigned t = xbeg(n); t < xend(n); t += xstride()) ux[t * (unsigned)g.fd[0][0]] = u_in;
}

// Back-to-back launches of one kernel family on the live state, between two
// events; *ms = average per launch.  The transport hierarchy (h = 3) stands for
// the V-cycle families; its buffers and the Krylov scratch vectors are only
// overwritten with values no later step reads.
template <typename R>
vos_status time_kernel_t(vos_sim *s, SLevel<R> *lv, int family, int reps, double *ms, double *bytes)
{
  hipStream_t st = s->stream;
  const Dev &g = s->g;
  const int nd = g.nd;
  const int L = s->snlev[3];
  int lc = 0;
  while (lc < L - 1 && lv[lc].nc > (unsigned)s->coarse_cells) ++lc;
  const double *flag = sc_block(s, SC_MISC) + S_COUNT;   // always unconverged
  const R om = (R)0.85;
  const double Rs = sizeof(R);
  // bytes of a level's 2 nd off-diagonals (FP32 copies where the level keeps them)
  auto offb = [&](int l) { return 2.0 * nd * (lv[l].off32 ? sizeof(float) : Rs); };
  double per_seq_bytes = 0.0;
  int per_seq_launches = 0;
  auto seq = [&](bool count) {
    switch (family) {
      case VOS_KERNEL_V_RESTRICT:
        for (int l = 0; l < lc; ++l) {
          k_v_restrict<SLevel<R>, R><<<grid_blocks(lv[l + 1].nc), TPB, 0, st>>>(lv[l], lv[l + 1], nd, flag);
          if (count) { per_seq_bytes += (3.0 * Rs + offb(l)) * lv[l].nc + Rs * lv[l + 1].nc; ++per_seq_launches; }
        }
        break;
      case VOS_KERNEL_V_POST:
        for (int l = 0; l < lc; ++l) {
          k_v_post<SLevel<R>, R, false><<<grid_blocks(lv[l].nc), TPB, 0, st>>>(lv[l], lv[l + 1], nd, lv[l].t, om,
                                                                               nullptr, nullptr, flag);
          if (count) { per_seq_bytes += (4.0 * Rs + offb(l)) * lv[l].nc + Rs * lv[l + 1].nc; ++per_seq_launches; }
        }
        break;
      case VOS_KERNEL_V_PRE:
        for (int l = 1; l < lc; ++l) {
          k_v_pre<SLevel<R>, R, false, 2><<<grid_blocks(lv[l].nc), TPB, 0, st>>>(lv[l], nd, nullptr, nullptr, 1.0,
                                                                                 om, flag);
          if (count) { per_seq_bytes += (3.0 * Rs + offb(l)) * lv[l].nc; ++per_seq_launches; }
        }
        break;
      case VOS_KERNEL_V_COARSE: {
        LevelPack<SLevel<R>> pack;
        for (int l = 0; l < L && l < VC_MAX_LEVELS; ++l) pack.lv[l] = lv[l];
        launch_coarse<SLevel<R>, R>(coarse_in_lds(lv, lc, L, nd, s->opt.level_kernels == 0), pack, lc, L, nd,
                                    sweeps(s, 3), om, s->sainv[3], flag, st);
        if (count) {
          for (int l = lc; l < L; ++l) per_seq_bytes += (5.0 + 2 * nd) * Rs * lv[l].nc;
          ++per_seq_launches;
        }
        break;
      }
      case VOS_KERNEL_V_DOWN:
      case VOS_KERNEL_V_UP: {
        // the tiled 2-D kernels of the finest level
        const int ty = tile_height(lv[0].nc, s->tile_big);
        const dim3 gr(tile_blocks(lv[0].n[0], lv[0].n[1], ty));
        const int nu = sweeps(s, 3);
        const SLevel<R> &F0 = lv[0], &F1 = lv[1];
#define TDOWN(NU_, TY_) k_v_down2d<SLevel<R>, R, false, NU_, TY_><<<gr, TPB, 0, st>>>(F0, F1, nullptr, nullptr, 1.0, om, flag)
#define TUP(NU_, TY_) k_v_up2d<SLevel<R>, R, false, NU_, TY_><<<gr, TPB, 0, st>>>(F0, F1, F0.t, om, nullptr, nullptr, flag)
        if (family == VOS_KERNEL_V_DOWN) {
          if (ty == VT_Y_BIG) {
            if (nu == 2) TDOWN(2, VT_Y_BIG); else if (nu == 3) TDOWN(3, VT_Y_BIG); else TDOWN(4, VT_Y_BIG);
          } else {
            if (nu == 2) TDOWN(2, VT_Y_SMALL); else if (nu == 3) TDOWN(3, VT_Y_SMALL); else TDOWN(4, VT_Y_SMALL);
          }
          if (count) { per_seq_bytes += (3.0 * Rs + offb(0)) * lv[0].nc + Rs * lv[1].nc; ++per_seq_launches; }
        } else {
          if (ty == VT_Y_BIG) {
            if (nu == 2) TUP(2, VT_Y_BIG); else if (nu == 3) TUP(3, VT_Y_BIG); else TUP(4, VT_Y_BIG);
          } else {
            if (nu == 2) TUP(2, VT_Y_SMALL); else if (nu == 3) TUP(3, VT_Y_SMALL); else TUP(4, VT_Y_SMALL);
          }
          if (count) { per_seq_bytes += (4.0 * Rs + offb(0)) * lv[0].nc + Rs * lv[1].nc; ++per_seq_launches; }
        }
#undef TDOWN
#undef TUP
        break;
      }
      case VOS_KERNEL_P_APPLY:
        p_apply(s, s->p, s->vec[4], flag);
        if (count) { per_seq_bytes += (2.0 + nd) * 8.0 * g.nc; ++per_seq_launches; }
        break;
      case VOS_KERNEL_ADR_APPLY:
        k_adr_apply<1><<<grid_blocks(g.nc), TPB, 0, st>>>(g, s->off, s->c, s->vec[7], s->c, s->part, flag);
        if (count) { per_seq_bytes += (3.0 + 2 * nd) * 8.0 * g.nc; ++per_seq_launches; }
        break;
    }
  };
  if (family < VOS_KERNEL_V_RESTRICT || family > VOS_KERNEL_V_UP) return fail(VOS_ERR_ARG, "unknown kernel family");
  if ((family == VOS_KERNEL_V_DOWN || family == VOS_KERNEL_V_UP) &&
      !(nd == 2 && sweeps(s, 3) >= 2 && sweeps(s, 3) <= 4 && lc >= 1 && lv[0].n[0] >= 2 && lv[0].n[1] >= 2))
    return fail(VOS_ERR_ARG, "the tiled V-cycle kernels run on 2-D levels with 2..4 sweeps only");
  seq(true);   // warm-up, counts the launches of one sequence
  if (per_seq_launches == 0) return fail(VOS_ERR_STATE, "the hierarchy has no level of that kind");
  HIP_TRY(hipEventRecord(s->ev[0], st));
  for (int k = 0; k < reps; ++k) seq(false);
  HIP_TRY(hipEventRecord(s->ev[1], st));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventSynchronize(s->ev[1]));
  float el = 0.f;
  HIP_TRY(hipEventElapsedTime(&el, s->ev[0], s->ev[1]));
  *ms = (double)el / ((double)reps * per_seq_launches);
  *bytes = per_seq_bytes / per_seq_launches;
  return VOS_OK;
}

}  // namespace

// Back-to-back launches of one z-marching kernel of a 3-D hierarchy's finest
// level with the production launch shape: the pressure hierarchy (in the
// arithmetic the last pressure solve used), the transport hierarchy (FP64) or
// the x-momentum hierarchy.  They write only the level's V-cycle buffers,
// which every V-cycle rebuilds from its input.  Bytes per fine cell, every
// array once (w = bytes of the hierarchy's arithmetic; cb = coefficient bytes
// per cell: 3 face arrays T for the pressure levels, whose finest diagonal is
// the sum of the faces, else the diagonal and 6 off-diagonals, these in FP32
// where the level keeps FP32 copies):
//   pre (first down launch, two sweeps from the FP64 residual): r (8) +
//     coefficients, write b, write x (cb + 2 w);
//   sweep: x, coefficients, b, write (cb + 3 w);
//   restrict: x, coefficients, b (cb + 2 w) + coarse b (w / 8);
//   post (prolongation + first up sweep): x, coefficients, b, write
//     (cb + 3 w) + coarse x (w / 8);
//   fused down leg (two sweeps from the FP64 residual and the restriction):
//     r (8) + coefficients, write x (cb + w) + coarse b (w / 8);
//   fused up leg (prolongation and two sweeps, FP64 output): x, coefficients
//     (cb + w), r (8), write (8) + coarse x (w / 8).
template <typename R>
double coef_bytes(const MgLevel<R> &) { return 3.0 * sizeof(R); }
template <typename R>
double coef_bytes(const SLevel<R> &L) { return sizeof(R) + 6.0 * (L.off32 ? sizeof(float) : sizeof(R)); }

template <typename Lv, typename R>
vos_status time_z_kernel_t(vos_sim *s, Lv *lv, int nlev, int kind, double omega, double rscale, int reps, double *ms,
                           double *bytes, bool rg = false)
{
  hipStream_t st = s->stream;
  if (s->g.nd != 3 || nlev < 2) return fail(VOS_ERR_ARG, "the z-marching level families time 3-D hierarchies");
  Lv F = lv[0];
  if (!(F.n[0] >= ZT_X / 2 && F.n[1] >= 2 && F.n[2] >= 2))
    return fail(VOS_ERR_ARG, "the finest level is too narrow for the z-marching kernels");
  const int zl = zrun_len(F.n);
  const dim3 gr(zrun_blocks(F.n, zl));
  if (kind >= 4 && !zfused_level(F.n)) return fail(VOS_ERR_ARG, "the fused legs run on levels of >= 2^20 cells");
  const double *flag = sc_block(s, SC_MISC) + S_COUNT;   // always unconverged
  const R om = (R)omega;
  const double w = sizeof(R), nc = F.nc, cb = coef_bytes(F);
  double per = 0.0;
  auto launch = [&]() {
    switch (kind) {
      case 0:
        k_v_pre3d<Lv, R, RHS_R><<<gr, TPB, 0, st>>>(F, s->vec[1], nullptr, rscale, om, zl, flag);
        per = (8.0 + cb + 2.0 * w) * nc;
        break;
      case 1:
        k_v_jacobi3d<Lv, R, false><<<gr, TPB, 0, st>>>(F, F.x, F.t, om, nullptr, nullptr, zl, flag);
        per = (cb + 3.0 * w) * nc;
        break;
      case 2:
        k_v_restrict3d<Lv, R><<<gr, TPB, 0, st>>>(F, lv[1], zl, flag);
        per = (cb + 2.0 * w) * nc + w * lv[1].nc;
        break;
      case 3:
        k_v_post3d<Lv, R, false><<<gr, TPB, 0, st>>>(F, lv[1], F.t, om, nullptr, nullptr, zl, flag);
        per = (cb + 3.0 * w) * nc + w * lv[1].nc;
        break;
      case 4:
        fused_down<Lv, R>(s, F, lv[1], true, s->vec[1], rscale, om, flag, st, rg);
        per = (8.0 + cb + w) * nc + w * lv[1].nc;
        break;
      default:
        fused_up<Lv, R>(s, F, lv[1], true, s->vec[2], s->vec[1], rscale, om, flag, st, rg);
        per = (cb + w + 16.0) * nc + w * lv[1].nc;
        break;
    }
  };
  launch();   // warm-up
  HIP_TRY(hipEventRecord(s->ev[0], st));
  for (int k = 0; k < reps; ++k) launch();
  HIP_TRY(hipEventRecord(s->ev[1], st));
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipEventSynchronize(s->ev[1]));
  float el = 0.f;
  HIP_TRY(hipEventElapsedTime(&el, s->ev[0], s->ev[1]));
  *ms = (double)el / reps;
  *bytes = per;
  return VOS_OK;
}

// Frees what vos_create made besides the workspace (the caller's); used on
// creation failure and by vos_destroy.
void release(vos_sim *s)
{
  for (int k = 0; k < 3; ++k)
    if (s->lane_stream[k]) (void)hipStreamSynchronize(s->lane_stream[k]);
  drop_graphs(s);
  for (int k = 0; k < 7; ++k)
    if (s->ev[k]) (void)hipEventDestroy(s->ev[k]);
  if (s->fork) (void)hipEventDestroy(s->fork);
  for (int k = 0; k < 3; ++k) {
    if (s->join[k]) (void)hipEventDestroy(s->join[k]);
    if (s->lane_stream[k]) (void)hipStreamDestroy(s->lane_stream[k]);
  }
  if (s->host) (void)hipHostFree(s->host);
  if (s->host2) (void)hipHostFree(s->host2);
  if (s->host3) (void)hipHostFree(s->host3);
  delete s;
}

// ====================================================================== C ABI

extern "C" {

const char *vos_last_error(void) { return g_err.c_str(); }

vos_status vos_workspace_bytes(const vos_grid *grid, const vos_opts *opts, size_t *bytes)
{
  vos_status st = check_grid(grid);
  if (st) return st;
  if ((st = check_opts(opts))) return st;
  if (!bytes) return fail(VOS_ERR_ARG, "bytes is NULL");
  *bytes = make_layout(*grid, opts->precision).total;
  return VOS_OK;
}

vos_status vos_create(const vos_grid *grid, const vos_params *params, const vos_opts *opts, void *workspace,
                      size_t workspace_bytes, void *hip_stream, vos_sim **out)
{
  vos_status st = check_grid(grid);
  if (st) return st;
  if ((st = check_params(params))) return st;
  if ((st = check_opts(opts))) return st;
  if ((st = check_combination(params, opts))) return st;
  if (!out) return fail(VOS_ERR_ARG, "out is NULL");
  if (!workspace || ((uintptr_t)workspace % ALIGN) != 0) return fail(VOS_ERR_ARG, "workspace must be 256-byte aligned");
  Layout lo = make_layout(*grid, opts->precision);
  if (workspace_bytes < lo.total) return fail(VOS_ERR_OOM, "workspace smaller than vos_workspace_bytes()");
  vos_sim *s = new (std::nothrow) vos_sim();
  if (!s) return fail(VOS_ERR_OOM, "host allocation failed");
  s->grid = *grid;
  s->prm = *params;
  s->opt = *opts;
  s->stream = (hipStream_t)hip_stream;
  s->n_cu = device_cus();
  s->lo = lo;
  s->ws = (char *)workspace;
  Dev &g = s->g;
  g.n[0] = grid->nx; g.n[1] = grid->ny; g.n[2] = grid->nz;
  g.nd = grid->nz == 1 ? 2 : 3;
  for (int d = 0; d < 3; ++d) {
    for (int e = 0; e < 3; ++e) g.fd[d][e] = g.n[e] + (e == d);
    g.nf[d] = (unsigned)g.fd[d][0] * g.fd[d][1] * g.fd[d][2];
  }
  g.nc = (unsigned)grid->nx * grid->ny * grid->nz;
  g.dx = grid->dx; g.S = grid->dx * grid->dx; g.V = g.S * grid->dx;
  g.drive = params->drive;
  Phys &P = s->P;
  fill_phys(P, params, *opts);
  char *w = s->ws;
  auto D = [&](size_t o) { return (double *)(w + o); };
  s->eps = D(lo.eps); s->p = D(lo.p); s->c = D(lo.c); s->pn = D(lo.pn); s->cold = D(lo.cold);
  for (int k = 0; k < NHIST; ++k) {
    s->cprev[k] = D(lo.cprev[k]);
    s->pprev[k] = D(lo.pprev[k]);
    for (int d = 0; d < 3; ++d) s->uprev[d][k] = D(lo.uprev[d][k]);
  }
  s->rbar = D(lo.rbar); s->gmag = D(lo.gmag); s->pdiag = D(lo.pdiag); s->off = D(lo.off);
  s->c0 = D(lo.c0); s->eps_prev = D(lo.eps_prev);
  s->tdiag = D(lo.tdiag); s->tdif = D(lo.tdif);
  for (int d = 0; d < 3; ++d) {
    s->nrm[d] = D(lo.nrm[d]); s->u[d] = D(lo.u[d]); s->ustar[d] = D(lo.ustar[d]); s->dmom[d] = D(lo.dmom[d]);
    s->af[d] = D(lo.af[d]); s->T[d] = D(lo.T[d]); s->w[d] = D(lo.w[d]);
  }
  for (int k = 0; k < NVEC; ++k) s->vec[k] = D(lo.vec[k]);
  s->part = D(lo.part); s->part_max = D(lo.part_max); s->scal = D(lo.scal); s->ainv = D(lo.ainv);
  s->nlev = lo.nlev;
  fill_levels<float>(s, s->mgf);
  fill_levels<double>(s, s->mgd);
  for (int h = 0; h < NSMG; ++h) {
    fill_smg<float>(s, h, s->smgf[h]);
    fill_smg<double>(s, h, s->smgd[h]);
  }
  s->have_geometry = false;
  s->stepped = false;
  s->net = nullptr;
  s->ws_gain = 1.0;
  s->ws_use = 0;
  s->ws_sampled = false;
  s->ws_s0 = 0.0;
  s->ws_used = 0;
  s->ws_res_prev = s->ws_res_guess = 0.0;
  s->it_p_fp64 = 0;
  s->p_fp64_sticky = false;
  s->hist_c = s->hist_p = 0;
  hierarchies_stale(s);
  s->hist_u[0] = s->hist_u[1] = s->hist_u[2] = 0;
  s->ws_drop = s->ws_frac = 0.0;
  std::memset(&s->last, 0, sizeof(s->last));
  s->part2 = D(lo.part2);
  s->part3 = D(lo.part3);
  s->host = s->host2 = s->host3 = nullptr;
  s->lane_stream[0] = s->lane_stream[1] = s->lane_stream[2] = nullptr;
  s->fork = s->join[0] = s->join[1] = s->join[2] = nullptr;
  for (int k = 0; k < 7; ++k) s->ev[k] = nullptr;
  hipError_t e = hipHostMalloc((void **)&s->host, 64 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&s->host2, 64 * sizeof(double), hipHostMallocDefault);
  if (e == hipSuccess) e = hipHostMalloc((void **)&s->host3, 64 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    release(s);
    return fail(VOS_ERR_DEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  // default priority; created back to back so they land on different hardware
  // queues (the sim's stream and three lanes: the four queues of a process)
  e = hipStreamCreateWithFlags(&s->lane_stream[0], hipStreamNonBlocking);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s->lane_stream[1], hipStreamNonBlocking);
  if (e == hipSuccess && s->g.nd == 3) e = hipStreamCreateWithFlags(&s->lane_stream[2], hipStreamNonBlocking);
  for (int k = 0; k < 7 && e == hipSuccess; ++k) e = hipEventCreate(&s->ev[k]);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&s->fork, hipEventDisableTiming);
  for (int k = 0; k < 3 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&s->join[k], hipEventDisableTiming);
  if (e != hipSuccess) {
    release(s);
    return fail(VOS_ERR_DEVICE, std::string("stream / event creation: ") + hipGetErrorString(e));
  }
  s->p_scale = 0.0;
  // defaults (0): a 1024-cell single-block tail in 2-D, 4096 cells in 3-D.
  // Sweeps: 2-D pressure 4 (fewer iterations at the same launch count); 3-D
  // pressure 3 (256^3 sphere pack to 1e-8: 564 iterations in 1.13 s, against
  // 2158 in 3.25 s with 2 and 500 in 1.25 s with 4); momentum 2 (measured
  // faster per step than 3 or 4 on the micromodel); transport at most 2
  if (s->opt.mg_nu == 0) s->opt.mg_nu = grid->nz == 1 ? 4 : 3;
  s->nu_mom = opts->mg_nu == 0 ? 2 : opts->mg_nu;
  s->coarse_cells = opts->coarse_cells > 0 ? opts->coarse_cells : (grid->nz == 1 ? VC_TAIL_2D : VC_BLOCK_MAX);
  s->tile_big = VT_BIG_CELLS;
  s->setup_every = std::max(1, opts->setup_every);
  s->use_graphs = opts->use_graphs != 0 && hip_stream != nullptr;   // the null stream cannot be captured
  for (int k = 0; k < 8; ++k) {
    s->gexec[k] = nullptr;
    s->last_its[k] = 0;
  }

  // initial state: fluid at rest, p = p_out, c = 0, eps = eps_prev = 1, no earlier rates
  hipStream_t stq = s->stream;
  HIP_TRY(hipMemsetAsync(s->ws, 0, lo.total, stq));
  k_fill<<<grid_blocks(g.nc), TPB, 0, stq>>>(g.nc, 1.0, s->eps);
  k_fill<<<grid_blocks(g.nc), TPB, 0, stq>>>(g.nc, 1.0, s->eps_prev);
  k_fill<<<grid_blocks(g.nc), TPB, 0, stq>>>(g.nc, P.p_out, s->p);
  k_inlet<<<grid_blocks((size_t)g.n[1] * g.n[2]), TPB, 0, stq>>>(g, inlet_velocity(s), s->u[0]);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(stq));
  *out = s;
  return VOS_OK;
}

vos_status vos_destroy(vos_sim *s)
{
  if (!s) return fail(VOS_ERR_ARG, "sim is NULL");
  (void)hipStreamSynchronize(s->stream);
  release(s);
  return VOS_OK;
}

vos_status vos_set_solid_fraction(vos_sim *s, const double *eps_s, int on_device)
{
  if (!s || !eps_s) return fail(VOS_ERR_ARG, "NULL argument");
  const Dev &g = s->g;
  hipStream_t st = s->stream;
  double *src = s->vec[0];
  HIP_TRY(hipMemcpyAsync(src, eps_s, g.nc * sizeof(double),
                         on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
  int *bad = (int *)(s->vec[1]);
  HIP_TRY(hipMemsetAsync(bad, 0, sizeof(int), st));
  k_set_eps<<<grid_blocks(g.nc), TPB, 0, st>>>(g.nc, src, s->P.eps_min, s->eps, bad);
  HIP_TRY(hipMemcpyAsync(s->eps_prev, s->eps, g.nc * sizeof(double), hipMemcpyDeviceToDevice, st));
  k_fill<<<grid_blocks(g.nc), TPB, 0, st>>>(g.nc, 0.0, s->rbar);
  s->p_fp64_sticky = false;   // a new geometry: mixed precision tries the FP32 hierarchy again
  s->hist_c = s->hist_p = 0;
  hierarchies_stale(s);
  s->hist_u[0] = s->hist_u[1] = s->hist_u[2] = 0;
  k_inlet<<<grid_blocks((size_t)g.n[1] * g.n[2]), TPB, 0, st>>>(g, inlet_velocity(s), s->u[0]);
  HIP_TRY(hipGetLastError());
  int hbad = 0;
  HIP_TRY(hipMemcpyAsync(s->host, bad, sizeof(int), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  std::memcpy(&hbad, s->host, sizeof(int));
  if (hbad) return fail(VOS_ERR_ARG, "solid fraction outside [0, 1]");
  s->have_geometry = true;
  return VOS_OK;
}

vos_status vos_set_params(vos_sim *s, const vos_params *params)
{
  if (!s) return fail(VOS_ERR_ARG, "sim is NULL");
  vos_status st = check_params(params);
  if (st) return st;
  if ((st = check_combination(params, &s->opt))) return st;
  s->prm = *params;
  drop_graphs(s);   // captured iterations hold mu / dx^2 by value
  s->hist_c = s->hist_p = 0;
  hierarchies_stale(s);
  s->hist_u[0] = s->hist_u[1] = s->hist_u[2] = 0;
  const int old_drive = s->g.drive;
  fill_phys(s->P, params, s->opt);
  s->g.drive = params->drive;
  // the velocity drive imposes u_in on the inlet faces; under the pressure drive
  // they are unknowns and keep their values (0 when switching from the velocity drive)
  if (params->drive == 0 || old_drive == 0)
    k_inlet<<<grid_blocks((size_t)s->g.n[1] * s->g.n[2]), TPB, 0, s->stream>>>(s->g, inlet_velocity(s), s->u[0]);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(s->stream));
  return VOS_OK;
}

vos_status vos_set_field(vos_sim *s, int field, const double *src, int on_device)
{
  if (!s || !src) return fail(VOS_ERR_ARG, "NULL argument");
  size_t n;
  bool wr;
  double *d = field_ptr(s, field, &n, &wr);
  if (!d) return fail(VOS_ERR_ARG, "unknown field");
  if (!wr) return fail(VOS_ERR_ARG, "field is read-only");
  s->hist_c = s->hist_p = 0;
  hierarchies_stale(s);
  s->hist_u[0] = s->hist_u[1] = s->hist_u[2] = 0;
  HIP_TRY(hipMemcpyAsync(d, src, n * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  if (field == VOS_FIELD_EPS) s->have_geometry = true;
  return VOS_OK;
}

vos_status vos_get_field(vos_sim *s, int field, double *dst, int on_device)
{
  if (!s || !dst) return fail(VOS_ERR_ARG, "NULL argument");
  size_t n;
  bool wr;
  double *d = field_ptr(s, field, &n, &wr);
  if (!d) return fail(VOS_ERR_ARG, "unknown field");
  HIP_TRY(hipMemcpyAsync(dst, d, n * sizeof(double), on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                         s->stream));
  HIP_TRY(hipStreamSynchronize(s->stream));
  return VOS_OK;
}

vos_status vos_field_ptr(vos_sim *s, int field, double **dev_ptr)
{
  if (!s || !dev_ptr) return fail(VOS_ERR_ARG, "NULL argument");
  size_t n;
  bool wr;
  double *d = field_ptr(s, field, &n, &wr);
  if (!d) return fail(VOS_ERR_ARG, "unknown field");
  *dev_ptr = d;
  return VOS_OK;
}

vos_status vos_step(vos_sim *s, double dt, int nsteps, int flags, vos_diag *last)
{
  if (!s) return fail(VOS_ERR_ARG, "sim is NULL");
  if (!(dt > 0.0) || nsteps < 0) return fail(VOS_ERR_ARG, "dt must be > 0 and nsteps >= 0");
  if (!s->have_geometry) return fail(VOS_ERR_STATE, "set the solid fraction before stepping");
  vos_diag dg;
  std::memset(&dg, 0, sizeof(dg));
  for (int k = 0; k < nsteps; ++k) {
    vos_status st = one_step(s, dt, flags, &dg);
    s->last = dg;
    s->stepped = true;
    if (st) {
      if (last) *last = dg;
      return st;
    }
  }
  if (last) *last = s->last;
  return VOS_OK;
}

vos_status vos_time_kernel(vos_sim *s, int family, int reps, double *avg_launch_ms, double *bytes_per_launch)
{
  if (!s || !avg_launch_ms || !bytes_per_launch) return fail(VOS_ERR_ARG, "NULL argument");
  if (reps < 1 || reps > 100000) return fail(VOS_ERR_ARG, "reps must be in [1, 100000]");
  if (!s->stepped) return fail(VOS_ERR_STATE, "run vos_step first");
  if (family >= VOS_KERNEL_P_PRE3D && family <= VOS_KERNEL_P_POST3D) {
    const int kind = family - VOS_KERNEL_P_PRE3D;
    if (s->opt.precision == VOS_MIXED && !s->p_fp64_sticky)
      return time_z_kernel_t<MgLevel<float>, float>(s, s->mgf, s->nlev, kind, 6.0 / 7.0, 1.0 / s->p_scale, reps,
                                                     avg_launch_ms, bytes_per_launch);
    return time_z_kernel_t<MgLevel<double>, double>(s, s->mgd, s->nlev, kind, 6.0 / 7.0, 1.0 / s->p_scale, reps,
                                                     avg_launch_ms, bytes_per_launch);
  }
  if (family == VOS_KERNEL_M_DOWN3D || family == VOS_KERNEL_M_UP3D) {
    const int kind = 4 + (family - VOS_KERNEL_M_DOWN3D);
    if (s->opt.precision == VOS_MIXED)
      return time_z_kernel_t<SLevel<float>, float>(s, s->smgf[0], s->snlev[0], kind, 0.85, 1.0, reps, avg_launch_ms,
                                                   bytes_per_launch);
    return time_z_kernel_t<SLevel<double>, double>(s, s->smgd[0], s->snlev[0], kind, 0.85, 1.0, reps, avg_launch_ms,
                                                   bytes_per_launch);
  }
  if (family >= VOS_KERNEL_C_PRE3D && family <= VOS_KERNEL_C_UP3D)
    return time_z_kernel_t<SLevel<double>, double>(s, s->smgd[3], s->snlev[3], family - VOS_KERNEL_C_PRE3D, 0.85, 1.0,
                                                    reps, avg_launch_ms, bytes_per_launch,
                                                    smg_finest_fused(s, 3, s->smgd[3]));
  return time_kernel_t<double>(s, s->smgd[3], family, reps, avg_launch_ms, bytes_per_launch);
}

vos_status vos_diagnostics(vos_sim *s, vos_diag *out)
{
  if (!s || !out) return fail(VOS_ERR_ARG, "NULL argument");
  *out = s->last;
  return VOS_OK;
}

vos_status vos_solve_pressure(vos_sim *s, double dt, const double *guess, int on_device, vos_diag *out)
{
  if (!s) return fail(VOS_ERR_ARG, "sim is NULL");
  if (!(dt > 0.0)) return fail(VOS_ERR_ARG, "dt must be > 0");
  if (!s->have_geometry) return fail(VOS_ERR_STATE, "set the solid fraction before solving");
  const Dev &g = s->g;
  hipStream_t st = s->stream;
  set_time_step(s, dt);
  launch_coefficients(s, dt);
  // the current face velocities are the predictor
  for (int d = 0; d < g.nd; ++d)
    HIP_TRY(hipMemcpyAsync(s->ustar[d], s->u[d], g.nf[d] * sizeof(double), hipMemcpyDeviceToDevice, st));
  const double *gs = nullptr;
  if (guess) {
    // staged in the history buffer the extrapolated starts use last (the
    // solve copies it into p after saving p^n); a caller's start ends that history
    double *buf = s->pprev[NHIST - 1];
    HIP_TRY(hipMemcpyAsync(buf, guess, g.nc * sizeof(double),
                           on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, st));
    gs = buf;
    s->hist_p = 0;
  }
  vos_diag dg;
  std::memset(&dg, 0, sizeof(dg));
  double r0 = 0.0;
  HIP_TRY(hipEventRecord(s->ev[2], st));
  vos_status rc = solve_pressure(s, &dg.it_p, &dg.res_p, &r0, gs);
  if (rc == VOS_ERR_DEVICE) return rc;
  HIP_TRY(hipEventRecord(s->ev[3], st));
  HIP_TRY(hipEventSynchronize(s->ev[3]));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, s->ev[2], s->ev[3]));
  dg.t_ms[2] = ms;
  dg.it_p_fp64 = s->it_p_fp64;
  dg.outer_res = r0;
  dg.outer_its = 1;
  s->stepped = true;
  if (out) *out = dg;
  return rc;
}

vos_status vos_initialize(vos_sim *s, double dt, int max_iters, double tol, vos_diag *out)
{
  if (!s) return fail(VOS_ERR_ARG, "sim is NULL");
  if (!(dt > 0.0) || max_iters < 1 || !(tol >= 0.0)) return fail(VOS_ERR_ARG, "need dt > 0, max_iters >= 1, tol >= 0");
  if (!s->have_geometry) return fail(VOS_ERR_STATE, "set the solid fraction before initializing");
  if (s->opt.simple) return fail(VOS_ERR_ARG, "vos_initialize relaxes the one-pass flow (simple = 0)");
  hipStream_t st = s->stream;
  const Dev &g = s->g;
  vos_diag dg;
  std::memset(&dg, 0, sizeof(dg));
  vos_status rc = VOS_OK;
  set_time_step(s, dt);
  launch_coefficients(s, dt);   // eps is frozen: the coefficients hold for every flow iteration
  // the face velocities before each iteration go to the oldest predictor history
  // buffers (the extrapolation history restarts afterwards anyway)
  double *prev[3] = {s->uprev[0][NHIST - 1], s->uprev[1][NHIST - 1], s->uprev[2][NHIST - 1]};
  double *sc = sc_block(s, SC_MISC) + 2;
  bool settled = false;
  for (int it = 0; it < max_iters; ++it) {
    for (int d = 0; d < g.nd; ++d)
      HIP_TRY(hipMemcpyAsync(prev[d], s->u[d], g.nf[d] * sizeof(double), hipMemcpyDeviceToDevice, st));
    double q = 0.0;
    if (vos_status e = momentum_stage(s, dt, &dg, &q, &rc)) return e;
    vos_status r2 = solve_pressure(s, &dg.it_p, &dg.res_p, &q);
    if (r2 == VOS_ERR_DEVICE) return r2;
    if (r2 && !rc) rc = r2;
    launch_correct(s);
    // relative change of the face velocities over the iteration
    for (int d = 0; d < g.nd; ++d)
      k_du<<<grid_blocks(g.nf[d]), TPB, 0, st>>>(g.nf[d], s->u[d], prev[d], s->part + 2 * d * MAXB);
    k_du_final<<<1, TPB, 0, st>>>(s->part, grid_blocks(g.nf[0]), grid_blocks(g.nf[1]),
                                  g.nd == 3 ? grid_blocks(g.nf[2]) : 0, sc);
    HIP_TRY(hipGetLastError());
    if (vos_status e = read_back(s, sc, 1)) return e;
    dg.outer_its = it + 1;
    dg.outer_res = s->host[0];
    if (rc) break;
    if (s->host[0] <= tol) { settled = true; break; }
  }
  s->hist_u[0] = s->hist_u[1] = s->hist_u[2] = 0;
  if (!rc) {
    // c^0: pure upwind, then one solve with the van Leer correction lagged on it
    double q = 0.0;
    vos_status r2 = solve_transport(s, dt, &dg.it_c, &dg.res_c, &q, 0);
    if (!r2) r2 = solve_transport(s, dt, &dg.it_c, &dg.res_c, &q, 1);
    if (r2 == VOS_ERR_DEVICE) return r2;
    if (r2 && !rc) rc = r2;
  }
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  s->stepped = true;
  if (out) *out = dg;
  if (rc) {
    std::string m = g_err;
    return fail(rc, m);
  }
  if (!settled) return fail(VOS_ERR_NOCONV, "the flow did not settle within max_iters");
  return VOS_OK;
}

// Checkpoint: a header of 8 64-bit words (magic, version, nx, ny, nz, field
// count, doubles that follow, 0) and the fields in a fixed order.
namespace {
constexpr uint64_t STATE_MAGIC = 0x564f5353544154ULL;   // "VOSSTAT"
constexpr uint64_t STATE_VERSION = 1;
constexpr int STATE_FIELDS = 8;

void state_fields(vos_sim *s, double *ptr[STATE_FIELDS], size_t n[STATE_FIELDS])
{
  const Dev &g = s->g;
  double *a[STATE_FIELDS] = {s->eps, s->eps_prev, s->rbar, s->u[0], s->u[1], s->u[2], s->p, s->c};
  const size_t m[STATE_FIELDS] = {g.nc, g.nc, g.nc, g.nf[0], g.nf[1], g.nf[2], g.nc, g.nc};
  for (int k = 0; k < STATE_FIELDS; ++k) { ptr[k] = a[k]; n[k] = m[k]; }
}

size_t state_doubles(vos_sim *s)
{
  double *ptr[STATE_FIELDS];
  size_t n[STATE_FIELDS], t = 0;
  state_fields(s, ptr, n);
  for (int k = 0; k < STATE_FIELDS; ++k) t += n[k];
  return t;
}
}  // namespace

vos_status vos_state_bytes(vos_sim *s, size_t *bytes)
{
  if (!s || !bytes) return fail(VOS_ERR_ARG, "NULL argument");
  *bytes = 8 * sizeof(uint64_t) + state_doubles(s) * sizeof(double);
  return VOS_OK;
}

vos_status vos_get_state(vos_sim *s, void *buf, size_t bytes)
{
  if (!s || !buf) return fail(VOS_ERR_ARG, "NULL argument");
  const size_t nd = state_doubles(s);
  if (bytes < 8 * sizeof(uint64_t) + nd * sizeof(double)) return fail(VOS_ERR_ARG, "state buffer too small");
  uint64_t *h = (uint64_t *)buf;
  h[0] = STATE_MAGIC; h[1] = STATE_VERSION;
  h[2] = (uint64_t)s->grid.nx; h[3] = (uint64_t)s->grid.ny; h[4] = (uint64_t)s->grid.nz;
  h[5] = STATE_FIELDS; h[6] = nd; h[7] = 0;
  double *ptr[STATE_FIELDS];
  size_t n[STATE_FIELDS];
  state_fields(s, ptr, n);
  char *dst = (char *)buf + 8 * sizeof(uint64_t);
  for (int k = 0; k < STATE_FIELDS; ++k) {
    HIP_TRY(hipMemcpyAsync(dst, ptr[k], n[k] * sizeof(double), hipMemcpyDeviceToHost, s->stream));
    dst += n[k] * sizeof(double);
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  return VOS_OK;
}

vos_status vos_set_state(vos_sim *s, const void *buf, size_t bytes)
{
  if (!s || !buf) return fail(VOS_ERR_ARG, "NULL argument");
  const size_t nd = state_doubles(s);
  if (bytes < 8 * sizeof(uint64_t)) return fail(VOS_ERR_ARG, "state buffer too small");
  const uint64_t *h = (const uint64_t *)buf;
  if (h[0] != STATE_MAGIC || h[1] != STATE_VERSION || h[5] != STATE_FIELDS)
    return fail(VOS_ERR_ARG, "not a state written by vos_get_state (or another version)");
  if (h[2] != (uint64_t)s->grid.nx || h[3] != (uint64_t)s->grid.ny || h[4] != (uint64_t)s->grid.nz || h[6] != nd)
    return fail(VOS_ERR_ARG, "the state belongs to another grid");
  if (bytes < 8 * sizeof(uint64_t) + nd * sizeof(double)) return fail(VOS_ERR_ARG, "state buffer truncated");
  double *ptr[STATE_FIELDS];
  size_t n[STATE_FIELDS];
  state_fields(s, ptr, n);
  const char *src = (const char *)buf + 8 * sizeof(uint64_t);
  for (int k = 0; k < STATE_FIELDS; ++k) {
    HIP_TRY(hipMemcpyAsync(ptr[k], src, n[k] * sizeof(double), hipMemcpyHostToDevice, s->stream));
    src += n[k] * sizeof(double);
  }
  HIP_TRY(hipStreamSynchronize(s->stream));
  s->hist_c = s->hist_p = 0;
  s->hist_u[0] = s->hist_u[1] = s->hist_u[2] = 0;
  hierarchies_stale(s);
  s->p_fp64_sticky = false;
  s->have_geometry = true;
  return VOS_OK;
}


vos_status vos_attach_unet(vos_sim *s, vos_unet *net, const vos_warm_start *ws)
{
  if (!s) return fail(VOS_ERR_ARG, "NULL simulation");
  if (!net) {
    s->net = nullptr;
    s->ws_use = 0;
    s->ws_sampled = false;
    return VOS_OK;
  }
  if (!ws) return fail(VOS_ERR_ARG, "NULL warm-start options");
  if (!(ws->gain > 0.0) || !std::isfinite(ws->gain)) return fail(VOS_ERR_ARG, "warm-start gain must be finite and > 0");
  int b, nz, ny, nx, cin;
  vosint::unet_dims(net, &b, &nz, &ny, &nx, &cin);
  if (b != 1 || nz != s->grid.nz || ny != s->grid.ny || nx != s->grid.nx || cin != 4)
    return fail(VOS_ERR_ARG, "the network must be planned for batch 1, the simulation's grid and 4 input channels");
  s->net = net;
  s->ws_gain = ws->gain;
  s->ws_use = ws->use_guess ? 1 : 0;
  s->ws_sampled = false;
  return VOS_OK;
}

vos_status vos_warm_start_sample(vos_sim *s, float *x_dev, float *target_dev)
{
  if (!s || !x_dev || !target_dev) return fail(VOS_ERR_ARG, "NULL argument");
  if (!s->net || !s->ws_sampled) return fail(VOS_ERR_STATE, "no pressure solve has run with a network attached");
  const unsigned n = s->g.nc;
  hipStream_t st = s->stream;
  HIP_TRY(hipMemcpyAsync(x_dev, vosint::unet_input(s->net), (size_t)n * 4 * sizeof(float), hipMemcpyDeviceToDevice,
                         st));
  k_ws_target<<<grid_blocks(n), TPB, 0, st>>>(n, s->p, s->pn, s->pdiag, s->ws_gain * s->ws_s0, target_dev);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(st));
  return VOS_OK;
}

}  // extern "C"

namespace vosint {

vos_status set_tuning(vos_sim *s, int check_every, int coarse_cells)
{
  if (!s) return fail(VOS_ERR_ARG, "NULL simulation");
  if (check_every < 1 || check_every > 256) return fail(VOS_ERR_ARG, "check_every must be in [1, 256]");
  if (coarse_cells != 0 && (coarse_cells < 64 || coarse_cells > 65536))
    return fail(VOS_ERR_ARG, "coarse_cells must be 0 or in [64, 65536]");
  drop_graphs(s);   // captured chunks hold the old chunk length and coarse split
  s->opt.check_every = check_every;
  s->opt.coarse_cells = coarse_cells;
  s->coarse_cells = coarse_cells > 0 ? coarse_cells : (s->g.nd == 2 ? VC_TAIL_2D : VC_BLOCK_MAX);
  return VOS_OK;
}

void get_tuning(const vos_sim *s, int *check_every, int *coarse_cells)
{
  *check_every = s->opt.check_every;
  *coarse_cells = s->opt.coarse_cells;
}

vos_status set_tile_big(vos_sim *s, unsigned cells)
{
  if (!s) return fail(VOS_ERR_ARG, "NULL simulation");
  if (cells < 1) return fail(VOS_ERR_ARG, "tile_big must be >= 1");
  if (cells != s->tile_big) drop_graphs(s);   // captured cycles hold the old tiles
  s->tile_big = cells;
  return VOS_OK;
}

unsigned get_tile_big(const vos_sim *s) { return s->tile_big; }

}  // namespace vosint

// ====================================================================== no-allocation pressure solve
//
// vos_solve_pressure_noalloc: the pressure equation of a state the caller
// passes in, with every scratch buffer (coefficients, Krylov vectors, the
// multigrid hierarchy, partial sums, solver scalars) carved from one
// file-scope device array instead of a caller workspace.  Host side it uses a
// control block and a read-back buffer of static storage, plain launches (no
// graph capture) and the caller's stream only.

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)48 << 20;   // 48 MiB per device
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES];   // device address of `scratch`, per device (null until looked up)
vos_sim g_noalloc_sim;                     // control block reused by every call of the process
double g_noalloc_host[64];                 // solver scalars read back here

// Offsets of the buffers the pressure stage needs within the scratch array:
// face coefficients (dmom, af, T), pressure diagonal, p^n, five Krylov vectors,
// partial sums, scalar blocks, the coarsest inverse and an FP64-sized hierarchy.
Layout pressure_layout(const vos_grid &g)
{
  Layout Lo;
  std::memset(&Lo, 0, sizeof(Lo));
  Plan P;
  LevelDims D0 = level_dims(g.nx, g.ny, g.nz);
  const size_t nc = D0.nc, dbl = sizeof(double);
  for (int d = 0; d < 3; ++d) {
    Lo.dmom[d] = P.take(D0.nf[d] * dbl);
    Lo.af[d] = P.take(D0.nf[d] * dbl);
    Lo.T[d] = P.take(D0.nf[d] * dbl);
  }
  Lo.pdiag = P.take(nc * dbl);
  Lo.pn = P.take(nc * dbl);
  for (int k = 0; k < 5; ++k) Lo.vec[k] = P.take(nc * dbl);
  Lo.part = P.take((size_t)NSLOT * MAXB * dbl);
  Lo.scal = P.take((size_t)NSC * S_COUNT * 2 * dbl);
  Lo.ainv = P.take((size_t)MG_COARSE_MAX * MG_COARSE_MAX * dbl);
  LevelDims lv[MG_MAX_LEVELS];
  Lo.nlev = mg_hierarchy(g, lv);
  for (int l = 0; l < Lo.nlev; ++l) {
    for (int d = 0; d < 3; ++d) Lo.mgT[l][d] = P.take(lv[l].nf[d] * dbl);
    Lo.mgdiag[l] = P.take(lv[l].nc * dbl);
    Lo.mgx[l] = P.take(lv[l].nc * dbl);
    Lo.mgb[l] = P.take(lv[l].nc * dbl);
    Lo.mgt[l] = P.take(lv[l].nc * dbl);
  }
  Lo.total = P.off;
  return Lo;
}

}  // namespace

extern "C" vos_status vos_solve_pressure_noalloc(const vos_grid *grid, const vos_params *params,
                                                 const vos_opts *opts, double dt, const double *eps,
                                                 const double *ux, const double *uy, const double *uz, double *p,
                                                 void *hip_stream, vos_diag *out)
{
  vos_status st = check_grid(grid);
  if (st) return st;
  if ((st = check_params(params))) return st;
  if ((st = check_opts(opts))) return st;
  if (!(dt > 0.0)) return fail(VOS_ERR_ARG, "dt must be > 0");
  const bool three = grid->nz > 1;
  if (!eps || !ux || !uy || !p || (three && !uz)) return fail(VOS_ERR_ARG, "NULL field pointer");
  if (params->transient) return fail(VOS_ERR_ARG, "the no-allocation pressure solve has no continuity source (transient = 0)");
  const Layout lo = pressure_layout(*grid);
  if (lo.total > NOALLOC_SCRATCH_BYTES)
    return fail(VOS_ERR_ARG, "grid too large for the no-allocation pressure solve: needs " + std::to_string(lo.total) +
                                 " bytes of scratch, the limit is " + std::to_string(NOALLOC_SCRATCH_BYTES));
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return fail(VOS_ERR_DEVICE, "device index beyond the supported range");
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(VOS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  char *base = (char *)g_scratch_ptr[dev];

  // the control block: the state's fields are the caller's, every other buffer is scratch
  vos_sim *s = &g_noalloc_sim;
  s->n_cu = device_cus();
  s->grid = *grid;
  s->prm = *params;
  s->opt = *opts;
  s->opt.extrapolate = 0;
  s->opt.simple = 0;
  s->stream = (hipStream_t)hip_stream;
  s->lo = lo;
  s->ws = base;
  Dev &g = s->g;
  g.n[0] = grid->nx; g.n[1] = grid->ny; g.n[2] = grid->nz;
  g.nd = three ? 3 : 2;
  g.drive = params->drive;
  for (int d = 0; d < 3; ++d) {
    for (int e = 0; e < 3; ++e) g.fd[d][e] = g.n[e] + (e == d);
    g.nf[d] = (unsigned)g.fd[d][0] * g.fd[d][1] * g.fd[d][2];
  }
  g.nc = (unsigned)grid->nx * grid->ny * grid->nz;
  g.dx = grid->dx; g.S = grid->dx * grid->dx; g.V = g.S * grid->dx;
  fill_phys(s->P, params, s->opt);
  auto D = [&](size_t o) { return (double *)(base + o); };
  s->eps = const_cast<double *>(eps);
  s->p = p;
  s->pn = D(lo.pn);
  s->pdiag = D(lo.pdiag);
  const double *uu[3] = {ux, uy, three ? uz : ux};
  for (int d = 0; d < 3; ++d) {
    s->dmom[d] = D(lo.dmom[d]); s->af[d] = D(lo.af[d]); s->T[d] = D(lo.T[d]);
    s->ustar[d] = const_cast<double *>(uu[d]);
    s->u[d] = s->ustar[d];
  }
  for (int k = 0; k < 5; ++k) s->vec[k] = D(lo.vec[k]);
  for (int k = 5; k < NVEC; ++k) s->vec[k] = nullptr;
  s->part = D(lo.part); s->scal = D(lo.scal); s->ainv = D(lo.ainv);
  s->rbar = nullptr;
  s->nlev = lo.nlev;
  fill_levels<float>(s, s->mgf);
  fill_levels<double>(s, s->mgd);
  s->host = g_noalloc_host;
  s->net = nullptr;
  s->ws_use = 0;
  s->use_graphs = false;
  for (int k = 0; k < 8; ++k) { s->gexec[k] = nullptr; s->last_its[k] = 0; }
  s->p_scale = 0.0;
  s->p_fp64_sticky = false;
  s->it_p_fp64 = 0;
  s->hist_p = 0;
  s->setup_every = 1;
  hierarchies_stale(s);
  if (s->opt.mg_nu == 0) s->opt.mg_nu = three ? 3 : 4;
  s->coarse_cells = opts->coarse_cells > 0 ? opts->coarse_cells : (three ? VC_BLOCK_MAX : VC_TAIL_2D);
  s->tile_big = VT_BIG_CELLS;

  hipStream_t stq = s->stream;
  // the scalar blocks hold the convergence flags and the always-zero flag: cleared per call
  k_fill<<<grid_blocks((size_t)NSC * S_COUNT * 2), TPB, 0, stq>>>((unsigned)(NSC * S_COUNT * 2), 0.0, s->scal);
  set_time_step(s, dt);
  k_face_coef<0><<<grid_blocks(g.nf[0]), TPB, 0, stq>>>(g, s->P, dt, s->eps, s->dmom[0], s->af[0], s->T[0]);
  k_face_coef<1><<<grid_blocks(g.nf[1]), TPB, 0, stq>>>(g, s->P, dt, s->eps, s->dmom[1], s->af[1], s->T[1]);
  if (three) k_face_coef<2><<<grid_blocks(g.nf[2]), TPB, 0, stq>>>(g, s->P, dt, s->eps, s->dmom[2], s->af[2], s->T[2]);
  else k_fill<<<grid_blocks(g.nf[2]), TPB, 0, stq>>>(g.nf[2], 0.0, s->T[2]);
  k_pdiag<<<grid_blocks(g.nc), TPB, 0, stq>>>(g, s->T[0], s->T[1], s->T[2], s->pdiag);
  vos_diag dg;
  std::memset(&dg, 0, sizeof(dg));
  double r0 = 0.0;
  vos_status rc = solve_pressure(s, &dg.it_p, &dg.res_p, &r0, nullptr);
  if (rc == VOS_ERR_DEVICE) return rc;
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipStreamSynchronize(stq));
  dg.it_p_fp64 = s->it_p_fp64;
  dg.outer_res = r0;
  dg.outer_its = 1;
  if (out) *out = dg;
  return rc;
}
