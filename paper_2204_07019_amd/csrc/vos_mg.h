// vos_mg.h -- cell-centred geometric multigrid V-cycle for the pressure
// equation, templated on the arithmetic of the hierarchy (float: the mixed
// mode; double: the FP64 mode).  Used as the preconditioner of FP64 flexible
// CG; it never decides convergence.
//
// Level l+1 halves every active dimension of level l.  Coarse transmissibility
// T_c = 1/2 * sum of the fine transmissibilities crossing the coarse face
// (parallel faces add, two fine cells in series halve it), which reproduces a
// rediscretisation on the coarse grid, including the outlet (Dirichlet) faces.
// Restriction sums the residual of the 2^nd children; prolongation is
// piecewise constant.  Smoother: damped Jacobi, nu sweeps before and after.
// The coarsest level (<= 64 cells) is solved with its dense inverse, rebuilt
// once per time step.
#pragma once
#include "vos_device.h"
#include "vos_kernels.h"

namespace vos {

constexpr int MG_MAX_LEVELS = 16;
constexpr int MG_COARSE_MAX = 64;

template <typename R>
struct MgLevel {
  int n[3];
  unsigned nc;
  unsigned nf[3];
  int fd[3][3];
  R *T[3];
  R *diag;
  R *x, *b, *t;
  // 1: diag is the sum of the cell's face coefficients in k_mg_diag's order
  // (the finest level), so a kernel that has loaded them may form it instead
  int dsum;
};

// A x at cell id.  Every load is issued unconditionally (a missing
// neighbour's index is clamped to the cell itself and its term skipped by a
// select), so all loads of a cell are in flight together; the arithmetic is
// the branchy form's: d x, then - T x per existing neighbour in slot order.
template <typename R>
__device__ __forceinline__ R mg_apply_cell(const MgLevel<R> &L, int nd, const R *x, unsigned id, const int c[3])
{
  const unsigned sy = (unsigned)L.n[0];
  const bool hw = c[0] > 0, he = c[0] < L.n[0] - 1, hs = c[1] > 0, hn = c[1] < L.n[1] - 1;
  const R xc = x[id];
  const R xw = x[hw ? id - 1 : id], xe = x[he ? id + 1 : id];
  const R xs = x[hs ? id - sy : id], xn = x[hn ? id + sy : id];
  const unsigned f0 = (unsigned)c[0] + (unsigned)L.fd[0][0] * ((unsigned)c[1] + (unsigned)L.fd[0][1] * c[2]);
  const R tw = L.T[0][f0], te = L.T[0][f0 + 1];
  const unsigned f1 = (unsigned)c[0] + (unsigned)L.fd[1][0] * ((unsigned)c[1] + (unsigned)L.fd[1][1] * c[2]);
  const R ts = L.T[1][f1], tn = L.T[1][f1 + L.fd[1][0]];
  R v = L.diag[id] * xc;
  v = hw ? v - tw * xw : v;
  v = he ? v - te * xe : v;
  v = hs ? v - ts * xs : v;
  v = hn ? v - tn * xn : v;
  if (nd == 3) {
    const unsigned sz = (unsigned)L.n[0] * L.n[1];
    const bool hb = c[2] > 0, ht = c[2] < L.n[2] - 1;
    const R xb = x[hb ? id - sz : id], xt = x[ht ? id + sz : id];
    const unsigned f2 = (unsigned)c[0] + (unsigned)L.fd[2][0] * ((unsigned)c[1] + (unsigned)L.fd[2][1] * c[2]);
    const R tb = L.T[2][f2], tt = L.T[2][f2 + sz];
    v = hb ? v - tb * xb : v;
    v = ht ? v - tt * xt : v;
  }
  return v;
}

// Level-0 diagonal: the sum of the cell's face transmissibilities (outlet included).
template <typename R>
__global__ void __launch_bounds__(TPB) k_mg_diag(MgLevel<R> L, int nd)
{
  for (unsigned id = xbeg(L.nc); id < xend(L.nc); id += xstride()) {
    int c[3];
    unflat(L.n, id, c);
    const unsigned f0 = (unsigned)c[0] + (unsigned)L.fd[0][0] * ((unsigned)c[1] + (unsigned)L.fd[0][1] * c[2]);
    const unsigned f1 = (unsigned)c[0] + (unsigned)L.fd[1][0] * ((unsigned)c[1] + (unsigned)L.fd[1][1] * c[2]);
    R s = L.T[0][f0] + L.T[0][f0 + 1] + L.T[1][f1] + L.T[1][f1 + L.fd[1][0]];
    if (nd == 3) {
      const unsigned f2 = (unsigned)c[0] + (unsigned)L.fd[2][0] * ((unsigned)c[1] + (unsigned)L.fd[2][1] * c[2]);
      s += L.T[2][f2] + L.T[2][f2 + (unsigned)L.n[0] * L.n[1]];
    }
    L.diag[id] = s;
  }
}

// Level 0 of the pressure hierarchy: T / s on every face (the outlet's
// Dirichlet face included), with one global scale s = the transmissibility of a
// fluid face (S dt / (rho dx)).  Raw coefficients span ~1e-30 (solid) to
// ~1e-13 (fluid); scaled, FP32 holds them and the residuals comfortably.  The
// scale is uniform so that piecewise-constant prolongation still acts on the
// unscaled pressure, which is continuous across the fluid-solid interface.
template <typename R, int D>
__global__ void __launch_bounds__(TPB) k_mg_scaled_faces(unsigned nf, const double *__restrict__ T, double inv_s,
                                                         MgLevel<R> L)
{
  for (unsigned f = xbeg(nf); f < xend(nf); f += xstride()) L.T[D][f] = (R)(T[f] * inv_s);
}

// Coarse diagonal, consistent with the coarse faces: the Galerkin diagonal of
// the aggregate times the rediscretisation factor 1/2,
// d_I = 1/2 [ sum_{c in I} d_c - 2 sum_{faces inside I} T ] = sum of the coarse faces' T.
template <typename R>
__global__ void __launch_bounds__(TPB) k_mg_coarse_diag(MgLevel<R> F, MgLevel<R> Cc, int nd)
{
  for (unsigned I = xbeg(Cc.nc); I < xend(Cc.nc); I += xstride()) {
    int X[3];
    unflat(Cc.n, I, X);
    R s = 0;
    const int lz = nd == 3 ? 2 : 1;
    for (int cz = 0; cz < lz; ++cz)
      for (int cy = 0; cy < 2; ++cy)
        for (int cx = 0; cx < 2; ++cx) {
          const int c[3] = {2 * X[0] + cx, 2 * X[1] + cy, nd == 3 ? 2 * X[2] + cz : 0};
          if ((F.n[0] == 1 && cx) || (F.n[1] == 1 && cy) || (cz && !(nd == 3 && F.n[2] > 1))) continue;
          if (c[0] >= F.n[0] || c[1] >= F.n[1] || c[2] >= F.n[2]) continue;
          const unsigned id = (unsigned)c[0] + (unsigned)F.n[0] * ((unsigned)c[1] + (unsigned)F.n[1] * (unsigned)c[2]);
          s += F.diag[id];
          // faces between this child and the next child of the same aggregate
          for (int d = 0; d < nd; ++d) {
            if (F.n[d] == 1 || (c[d] & 1) || c[d] + 1 >= F.n[d]) continue;
            int f[3] = {c[0], c[1], c[2]};
            f[d] += 1;
            const unsigned fi =
                (unsigned)f[0] + (unsigned)F.fd[d][0] * ((unsigned)f[1] + (unsigned)F.fd[d][1] * (unsigned)f[2]);
            s -= (R)2 * F.T[d][fi];
          }
        }
    Cc.diag[I] = (R)0.5 * s;
  }
}

// Coarse face transmissibilities of direction D from the fine level
// (ceil aggregation: the boundary face of an odd-sized level maps to the
// fine boundary face).
template <typename R, int D>
__global__ void __launch_bounds__(TPB) k_mg_coarsen(MgLevel<R> F, MgLevel<R> Cc, int nd)
{
  for (unsigned f = xbeg(Cc.nf[D]); f < xend(Cc.nf[D]); f += xstride()) {
    int X[3];
    unflat(Cc.fd[D], f, X);
    int x0[3];
    for (int e = 0; e < 3; ++e) x0[e] = (e < nd && F.n[e] > 1) ? 2 * X[e] : X[e];
    if (x0[D] > F.n[D]) x0[D] = F.n[D];
    R s = 0;
    const int c1 = (1 < nd && D != 1 && F.n[1] > 1) ? 2 : 1;
    const int c2 = (2 < nd && D != 2 && F.n[2] > 1) ? 2 : 1;
    const int c0 = (D != 0 && F.n[0] > 1) ? 2 : 1;
    for (int a = 0; a < c0; ++a)
      for (int bq = 0; bq < c1; ++bq)
        for (int cq = 0; cq < c2; ++cq) {
          const int i = x0[0] + a, j = x0[1] + bq, k = x0[2] + cq;
          if ((D != 0 && i >= F.n[0]) || (D != 1 && j >= F.n[1]) || (D != 2 && k >= F.n[2])) continue;
          s += F.T[D][(unsigned)i + (unsigned)F.fd[D][0] * ((unsigned)j + (unsigned)F.fd[D][1] * (unsigned)k)];
        }
    Cc.T[D][f] = (R)0.5 * s;
  }
}

// Dense inverse of the coarsest operator (n <= 64), FP64, one block: build
// A, scale to unit diagonal, Gauss-Jordan in place (SPD: no pivoting), unscale.
template <typename R>
__global__ void __launch_bounds__(GJ_TPB) k_mg_coarse_inverse(MgLevel<R> L, int nd, double *__restrict__ Ainv)
{
  __shared__ double M[MG_COARSE_MAX][MG_COARSE_MAX + 1];
  __shared__ double sc[MG_COARSE_MAX];
  const int n = (int)L.nc;
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) M[e / n][e % n] = 0.0;
  __syncthreads();
  for (int id = threadIdx.x; id < n; id += blockDim.x) {
    int c[3];
    unflat(L.n, (unsigned)id, c);
    M[id][id] = (double)L.diag[id];
    const unsigned f0 = (unsigned)c[0] + (unsigned)L.fd[0][0] * ((unsigned)c[1] + (unsigned)L.fd[0][1] * c[2]);
    const unsigned f1 = (unsigned)c[0] + (unsigned)L.fd[1][0] * ((unsigned)c[1] + (unsigned)L.fd[1][1] * c[2]);
    if (c[0] > 0) M[id][id - 1] = -(double)L.T[0][f0];
    if (c[0] < L.n[0] - 1) M[id][id + 1] = -(double)L.T[0][f0 + 1];
    if (c[1] > 0) M[id][id - L.n[0]] = -(double)L.T[1][f1];
    if (c[1] < L.n[1] - 1) M[id][id + L.n[0]] = -(double)L.T[1][f1 + L.fd[1][0]];
    if (nd == 3) {
      const int sz = L.n[0] * L.n[1];
      const unsigned f2 = (unsigned)c[0] + (unsigned)L.fd[2][0] * ((unsigned)c[1] + (unsigned)L.fd[2][1] * c[2]);
      if (c[2] > 0) M[id][id - sz] = -(double)L.T[2][f2];
      if (c[2] < L.n[2] - 1) M[id][id + sz] = -(double)L.T[2][f2 + sz];
    }
    sc[id] = 1.0 / sqrt((double)L.diag[id]);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    M[i][j] *= sc[i] * sc[j];
  }
  __syncthreads();
  {
    __shared__ double rowk[2][64], colk[2][64];
    gauss_jordan_inverse(M, n, rowk, colk);
  }
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e % n;
    Ainv[e] = M[i][j] * sc[i] * sc[j];
  }
}

}  // namespace vos
