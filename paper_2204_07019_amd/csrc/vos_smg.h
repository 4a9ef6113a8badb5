// vos_smg.h -- aggregation multigrid on explicit 7-point stencils, used to
// precondition the momentum (flexible CG) and transport (right-preconditioned
// BiCGStab) solves.  Templated on the arithmetic of the hierarchy.
//
// Level l+1 aggregates 2 cells per active dimension of level l (ceil, so odd
// sizes keep a one-cell aggregate at the end).  The coarse operator is the
// Galerkin product P^T A P with piecewise-constant P: couplings between two
// aggregates add up, couplings inside an aggregate fold into the diagonal.
// For the upwind transport operator this keeps the flux balance of every
// aggregate exact.  Restriction sums the children's residuals, prolongation
// injects.  Smoother: damped Jacobi.  Coarsest level (<= 64 cells): dense
// inverse built once per solve.
#pragma once
#include "vos_device.h"
#include "vos_kernels.h"

namespace vos {

constexpr int SMG_MAX_LEVELS = 20;
constexpr int SMG_COARSE_MAX = 64;

template <typename R>
struct SLevel {
  int n[3];
  unsigned nc;
  R *off;    // 6 * nc: -x, +x, -y, +y, -z, +z
  R *diag;
  R *x, *b, *t;
  R *dif;    // transport only (else nullptr): the diffusive part of each off-diagonal, 6 * nc
  // FP32 copies of off (6 * nc) that the smoother and the cycle's residuals read
  // instead, or nullptr.  Set on the levels of >= 2^20 cells of the 3-D
  // transport hierarchy in mixed precision: arithmetic, the diagonal and the
  // Galerkin products (which read off) stay FP64.
  float *off32;
};

// Off-diagonal of cell id towards neighbour slot k as the cycle's smoothing
// and residual arithmetic reads it.
template <typename R>
__device__ __forceinline__ R smg_off(const SLevel<R> &L, int k, unsigned id)
{
  if (L.off32) return (R)L.off32[(size_t)k * L.nc + id];
  return L.off[(size_t)k * L.nc + id];
}

// Piecewise-constant aggregation counts every diffusive coupling across a
// coarse face from all the fine faces it covers, twice what the diffusion
// operator rediscretised on the coarse cells holds (2-D: 2 faces of T each
// against T; 3-D: 4 against 2 T), so its coarse-grid corrections of smooth
// error come out half as large as they should.  The transport hierarchy keeps
// the diffusive part of every coupling apart and scales it by this factor on
// each coarser level; the advective and reactive parts (whose Galerkin sums
// are the coarse fluxes) stay as they are.
constexpr double SMG_DIFF_SCALE = 0.5;

// A x at cell id, every load issued unconditionally (as mg_apply_cell):
// d x, then + off x per existing neighbour in slot order.
template <typename R>
__device__ __forceinline__ R smg_apply_cell(const SLevel<R> &L, int nd, const R *x, unsigned id, const int c[3])
{
  const unsigned sy = (unsigned)L.n[0];
  const bool hw = c[0] > 0, he = c[0] < L.n[0] - 1, hs = c[1] > 0, hn = c[1] < L.n[1] - 1;
  const R xc = x[id];
  const R xw = x[hw ? id - 1 : id], xe = x[he ? id + 1 : id];
  const R xs = x[hs ? id - sy : id], xn = x[hn ? id + sy : id];
  const R ow = smg_off(L, 0, id), oe = smg_off(L, 1, id), os = smg_off(L, 2, id), on = smg_off(L, 3, id);
  R v = L.diag[id] * xc;
  v = hw ? v + ow * xw : v;
  v = he ? v + oe * xe : v;
  v = hs ? v + os * xs : v;
  v = hn ? v + on * xn : v;
  if (nd == 3) {
    const unsigned sz = (unsigned)L.n[0] * L.n[1];
    const bool hb = c[2] > 0, ht = c[2] < L.n[2] - 1;
    const R xb = x[hb ? id - sz : id], xt = x[ht ? id + sz : id];
    const R ob = smg_off(L, 4, id), ot = smg_off(L, 5, id);
    v = hb ? v + ob * xb : v;
    v = ht ? v + ot * xt : v;
  }
  return v;
}

// Level 0 of the transport hierarchy: the stencil without its row scaling
// (off64 is scaled by the diagonal dg; dif64 holds the unscaled diffusive
// parts), so the Galerkin products below are those of the operator itself.
// Where the level keeps FP32 copies of its off-diagonals (its smoothing reads
// only those), the FP64 ones are not stored: the Galerkin product forms them
// from off64 and dg itself (k_smg_coarsen's L0 form).  Where the level's
// diffusive parts are dif64 itself (3-D: every slot of dif64 is written),
// they are not copied.
// Damped Jacobi does not see a row scaling, so level 0 smooths as the scaled
// operator would; the cycle's input is the scaled residual times dg.
template <typename R>
__global__ void __launch_bounds__(TPB) k_smg_from_transport(unsigned nc, int nd, const double *__restrict__ off64,
                                                            const double *__restrict__ dg,
                                                            const double *__restrict__ dif64, SLevel<R> L)
{
  for (unsigned id = xbeg(nc); id < xend(nc); id += xstride()) {
    const double d = dg[id];
    L.diag[id] = (R)d;
    for (int k = 0; k < 6; ++k) {
      const bool on = k < 2 * nd;
      const double o = mul_rounded(off64[(size_t)k * nc + id], d);
      if (L.off32) L.off32[(size_t)k * nc + id] = on ? (float)o : 0.0f;
      else L.off[(size_t)k * nc + id] = on ? (R)o : (R)0;
      if ((const void *)L.dif != (const void *)dif64) L.dif[(size_t)k * nc + id] = on ? (R)dif64[(size_t)k * nc + id] : (R)0;
    }
  }
}

// Level 0 of the momentum hierarchy of component D on its face grid: the
// operator itself (diagonal dmom, -mu/dx^2 towards unknown neighbours; fixed
// rows identity).  Every coupling is viscous, so all of it is diffusive.
template <typename R, int D>
__global__ void __launch_bounds__(TPB) k_smg_from_momentum(Dev g, double cvis, const double *__restrict__ dmom,
                                                           SLevel<R> L)
{
  const unsigned nc = L.nc;
  for (unsigned f = xbeg(nc); f < xend(nc); f += xstride()) {
    int x[3];
    unflat(g.fd[D], f, x);
    L.diag[f] = (R)dmom[f];
    const bool unk = mom_unknown<D>(g, x);
    double fv;
    for (int e = 0; e < 3; ++e)
      for (int s = -1; s <= 1; s += 2) {
        const int slot = 2 * e + (s > 0);
        R v = 0;
        if (unk && e < g.nd && mom_nb<D>(g, x, e, s, 0.0, &fv) == 0) v = (R)(-cvis);
        L.off[(size_t)slot * nc + f] = v;
        L.dif[(size_t)slot * nc + f] = v;
      }
  }
}

// Galerkin coarse stencil of aggregate I.  L0: F is the transport
// hierarchy's level 0 whose FP64 off-diagonals are not stored; they are
// formed as k_smg_from_transport forms them, off64 times dg64.  With diffusive parts (F.dif), the
// coarse one is SMG_DIFF_SCALE times their Galerkin sum; the diffusion
// operator has zero row sums, so the diagonal drops by the same amount.  Per
// plane of children (one in 2-D, two in 3-D) every load is issued first, at
// clamped cells, and a missing child or neighbour is dropped by a select.
template <typename R, int ND, bool L0 = false>
__global__ void __launch_bounds__(TPB) k_smg_coarsen(SLevel<R> F, SLevel<R> C, const double *__restrict__ off64 = nullptr,
                                                     const double *__restrict__ dg64 = nullptr)
{
  constexpr int NS = 2 * ND;
  const bool split = F.dif != nullptr;
  const R *difs = split ? F.dif : F.off;   // read either way, used only when split
  for (unsigned I = xbeg(C.nc); I < xend(C.nc); I += xstride()) {
    int X[3];
    unflat(C.n, I, X);
    R dg = 0, o[6] = {0, 0, 0, 0, 0, 0}, q[6] = {0, 0, 0, 0, 0, 0};
#pragma unroll
    for (int cz = 0; cz < (ND == 3 ? 2 : 1); ++cz) {
      unsigned id[4];
      bool ok[4];
      int cc[4][3];
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        const int cx = ch & 1, cy = ch >> 1;
        const int c[3] = {2 * X[0] + cx, 2 * X[1] + cy, ND == 3 ? 2 * X[2] + cz : 0};
        // a dimension of extent 1 is not aggregated
        ok[ch] = c[0] < F.n[0] && c[1] < F.n[1] && c[2] < F.n[2] &&
                 !((F.n[1] == 1 && cy) || (ND == 3 && F.n[2] == 1 && cz) || (F.n[0] == 1 && cx));
        for (int e = 0; e < 3; ++e) cc[ch][e] = min(c[e], F.n[e] - 1);
        id[ch] = (unsigned)cc[ch][0] + (unsigned)F.n[0] * ((unsigned)cc[ch][1] + (unsigned)F.n[1] * cc[ch][2]);
      }
      R dv[4], av[4][NS], qv[4][NS];
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        dv[ch] = F.diag[id[ch]];
        const double d64 = L0 ? dg64[id[ch]] : 0.0;
#pragma unroll
        for (int k = 0; k < NS; ++k) {
          if constexpr (L0) av[ch][k] = (R)mul_rounded(off64[(size_t)k * F.nc + id[ch]], d64);
          else av[ch][k] = F.off[(size_t)k * F.nc + id[ch]];
          qv[ch][k] = difs[(size_t)k * F.nc + id[ch]];
        }
      }
#pragma unroll
      for (int ch = 0; ch < 4; ++ch) {
        dg = ok[ch] ? dg + dv[ch] : dg;
#pragma unroll
        for (int d = 0; d < ND; ++d) {
          const int cd = cc[ch][d];
          const int half = (F.n[d] == 1) ? 0 : 1;   // aggregated in this dimension?
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            const int k = 2 * d + s;
            const int nbc = s ? cd + 1 : cd - 1;
            const bool has = ok[ch] && nbc >= 0 && nbc < F.n[d];
            const bool inside = (half ? (cd >> 1) : cd) == (half ? (nbc >> 1) : nbc);
            const R a = av[ch][k], a_d = split ? qv[ch][k] : (R)0;
            dg = (has && inside) ? dg + a : dg;
            o[k] = (has && !inside) ? o[k] + a : o[k];
            q[k] = (has && !inside) ? q[k] + a_d : q[k];
          }
        }
      }
    }
    if (split) {
      const R keep = (R)(1.0 - SMG_DIFF_SCALE);
      for (int k = 0; k < 6; ++k) {
        o[k] -= keep * q[k];
        dg += keep * q[k];
        C.dif[(size_t)k * C.nc + I] = (R)SMG_DIFF_SCALE * q[k];
      }
    }
    C.diag[I] = dg;
    for (int k = 0; k < 6; ++k) C.off[(size_t)k * C.nc + I] = o[k];
    if (C.off32)
      for (int k = 0; k < 6; ++k) C.off32[(size_t)k * C.nc + I] = (float)o[k];
  }
}

// Dense inverse of the coarsest operator (n <= 64), FP64, one block.  Rows are
// scaled by the diagonal first (M = D^-1 A); the operators here are
// diagonally dominant, so Gauss-Jordan needs no pivoting; Ainv = M^-1 D^-1.
template <typename R>
__global__ void __launch_bounds__(GJ_TPB) k_smg_coarse_inverse(SLevel<R> L, int nd, double *__restrict__ Ainv)
{
  __shared__ double M[SMG_COARSE_MAX][SMG_COARSE_MAX + 1];
  __shared__ double rs[SMG_COARSE_MAX];
  const int n = (int)L.nc;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e / n][e % n] = 0.0;
  __syncthreads();
  for (int id = threadIdx.x; id < n; id += blockDim.x) {
    int c[3];
    unflat(L.n, (unsigned)id, c);
    const double dgl = (double)L.diag[id];
    rs[id] = 1.0 / dgl;
    M[id][id] = 1.0;
    const int sy = L.n[0], sz = L.n[0] * L.n[1];
    if (c[0] > 0) M[id][id - 1] = (double)L.off[id] / dgl;
    if (c[0] < L.n[0] - 1) M[id][id + 1] = (double)L.off[n + id] / dgl;
    if (c[1] > 0) M[id][id - sy] = (double)L.off[2 * n + id] / dgl;
    if (c[1] < L.n[1] - 1) M[id][id + sy] = (double)L.off[3 * n + id] / dgl;
    if (nd == 3) {
      if (c[2] > 0) M[id][id - sz] = (double)L.off[4 * n + id] / dgl;
      if (c[2] < L.n[2] - 1) M[id][id + sz] = (double)L.off[5 * n + id] / dgl;
    }
  }
  __syncthreads();
  {
    __shared__ double rowk[2][64], colk[2][64];
    gauss_jordan_inverse(M, n, rowk, colk);
  }
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    Ainv[e] = M[i][j] * rs[j];
  }
}

}  // namespace vos
