// vos_vcycle.h -- V-cycle kernels shared by the pressure hierarchy (MgLevel:
// face transmissibilities) and the momentum / transport hierarchies (SLevel:
// explicit stencils).  The level type only changes how A x is evaluated.
//
// Launch structure of one V-cycle, chosen for a latency-bound regime (each
// launch costs a few microseconds regardless of its size):
//  * fine levels (> VC_BLOCK_MAX cells), per level: one pre-smoothing kernel
//    (the first two damped-Jacobi sweeps fused: the first sweep from zero is
//    x1 = w b / d, evaluated on the fly at the neighbours), further sweeps if
//    nu > 2, one residual-restriction kernel, and on the way up one kernel
//    that fuses the prolongation with the first post-smoothing sweep, plus
//    the remaining sweeps;
//  * every level at or below VC_BLOCK_MAX cells runs inside ONE single-block
//    kernel (down-sweep, coarsest solve, up-sweep; __syncthreads between
//    phases), so the coarse tail costs one launch instead of ~6 per level.
// Aggregation is 2 cells per active dimension (ceil); a dimension of extent 1
// is not aggregated.
#pragma once
#include "vos_device.h"
#include "vos_kernels.h"
#include "vos_mg.h"
#include "vos_smg.h"

namespace vos {

constexpr int VC_BLOCK_MAX = 4096;   // levels at or below this size run in the single-block kernel
constexpr int VC_MAX_LEVELS = 20;
constexpr int VC_COARSE_TPB = 1024;

template <typename R>
__device__ __forceinline__ R lv_apply(const MgLevel<R> &L, int nd, const R *x, unsigned id, const int c[3])
{
  return mg_apply_cell(L, nd, x, id, c);
}

template <typename R>
__device__ __forceinline__ R lv_apply(const SLevel<R> &L, int nd, const R *x, unsigned id, const int c[3])
{
  return smg_apply_cell(L, nd, x, id, c);
}

// A x with x = x0 + xc[parent] (prolongation applied on the fly).
template <typename R>
__device__ __forceinline__ unsigned parent_of(const int fn[3], const int cn[3], int nd, const int c[3])
{
  const int I0 = fn[0] == 1 ? 0 : (c[0] >> 1);
  const int I1 = fn[1] == 1 ? 0 : (c[1] >> 1);
  const int I2 = (nd == 3 && fn[2] > 1) ? (c[2] >> 1) : 0;
  return (unsigned)I0 + (unsigned)cn[0] * ((unsigned)I1 + (unsigned)cn[1] * (unsigned)I2);
}

// The neighbours of cell id (up to 6), with their coordinates: calls f(nid, slot).
template <typename F>
__device__ __forceinline__ void for_neighbours(const int n[3], int nd, unsigned id, const int c[3], F &&f)
{
  const unsigned sy = (unsigned)n[0], sz = (unsigned)n[0] * n[1];
  if (c[0] > 0) f(id - 1, 0);
  if (c[0] < n[0] - 1) f(id + 1, 1);
  if (c[1] > 0) f(id - sy, 2);
  if (c[1] < n[1] - 1) f(id + sy, 3);
  if (nd == 3) {
    if (c[2] > 0) f(id - sz, 4);
    if (c[2] < n[2] - 1) f(id + sz, 5);
  }
}

// Off-diagonal coefficient of cell id towards neighbour slot k, for either level type.
template <typename R>
__device__ __forceinline__ R lv_off(const SLevel<R> &L, unsigned id, const int c[3], int k)
{
  (void)c;
  return L.off[(size_t)k * L.nc + id];
}

template <typename R>
__device__ __forceinline__ R lv_off(const MgLevel<R> &L, unsigned id, const int c[3], int k)
{
  (void)id;
  const int d = k >> 1;
  const int hi = k & 1;
  int f[3] = {c[0], c[1], c[2]};
  f[d] += hi;
  const unsigned fi = (unsigned)f[0] + (unsigned)L.fd[d][0] * ((unsigned)f[1] + (unsigned)L.fd[d][1] * (unsigned)f[2]);
  return -L.T[d][fi];
}

// ------------------------------------------------------------------ fine-level kernels

// Pre-smoothing, sweeps 1 and 2 fused.  FROM64: b = (R)(rscale r / sqrt(dsc)) on
// level 0 (dsc = diagonal of a symmetrically scaled operator, or nullptr;
// rscale = 1 / the global scale of an operator scaled by a constant).
// NSW = 1: only x = w b / d;  NSW = 2: x = x1 + w (b - A x1) / d with x1 = w b / d.
template <typename Lv, typename R, bool FROM64, int NSW>
__global__ void __launch_bounds__(TPB) k_v_pre(Lv L, int nd, const double *__restrict__ r64,
                                               const double *__restrict__ dsc, double rscale, R omega,
                                               const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  for (unsigned id = xbeg(L.nc); id < xend(L.nc); id += xstride()) {
    R bb;
    if (FROM64) bb = (R)(rscale * (dsc ? r64[id] / sqrt(dsc[id]) : r64[id]));
    else bb = L.b[id];
    if (FROM64) L.b[id] = bb;
    const R dg = L.diag[id];
    const R x1 = omega * bb / dg;
    if (NSW == 1) { L.x[id] = x1; continue; }
    int c[3];
    unflat(L.n, id, c);
    R ax = dg * x1;
    for_neighbours(L.n, nd, id, c, [&](unsigned nid, int k) {
      R bn;
      if (FROM64) bn = (R)(rscale * (dsc ? r64[nid] / sqrt(dsc[nid]) : r64[nid]));
      else bn = L.b[nid];
      ax += lv_off(L, id, c, k) * (omega * bn / L.diag[nid]);
    });
    L.x[id] = x1 + omega * (bb - ax) / dg;
  }
}

// FP64 output of level 0: z = x / sqrt(dsc) (or x when dsc is nullptr).
__device__ __forceinline__ double unscale(double v, const double *dsc, unsigned id)
{
  return dsc ? v / sqrt(dsc[id]) : v;
}

// One damped-Jacobi sweep xo = x + w (b - A x)/d; OUT64 also writes the FP64 result.
template <typename Lv, typename R, bool OUT64>
__global__ void __launch_bounds__(TPB) k_v_jacobi(Lv L, int nd, const R *__restrict__ x, R *__restrict__ xo, R omega,
                                                  double *__restrict__ z, const double *__restrict__ dsc,
                                                  const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  for (unsigned id = xbeg(L.nc); id < xend(L.nc); id += xstride()) {
    int c[3];
    unflat(L.n, id, c);
    const R v = x[id] + omega * (L.b[id] - lv_apply(L, nd, x, id, c)) / L.diag[id];
    xo[id] = v;
    if (OUT64) z[id] = unscale((double)v, dsc, id);
  }
}

// Coarse right-hand side: the fine residual summed over each aggregate.
template <typename Lv, typename R>
__device__ __forceinline__ R lv_restrict_one(const Lv &F, int nd, const int X[3])
{
  R s = 0;
  const int lz = nd == 3 ? 2 : 1;
  for (int cz = 0; cz < lz; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        const int c[3] = {F.n[0] == 1 ? 0 : 2 * X[0] + cx, F.n[1] == 1 ? 0 : 2 * X[1] + cy,
                          (nd == 3 && F.n[2] > 1) ? 2 * X[2] + cz : 0};
        if ((F.n[0] == 1 && cx) || (F.n[1] == 1 && cy) || (cz && !(nd == 3 && F.n[2] > 1))) continue;
        if (c[0] >= F.n[0] || c[1] >= F.n[1] || c[2] >= F.n[2]) continue;
        const unsigned id = (unsigned)c[0] + (unsigned)F.n[0] * ((unsigned)c[1] + (unsigned)F.n[1] * (unsigned)c[2]);
        s += F.b[id] - lv_apply(F, nd, F.x, id, c);
      }
  return s;
}

template <typename Lv, typename R>
__global__ void __launch_bounds__(TPB) k_v_restrict(Lv F, Lv C, int nd, const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  for (unsigned I = xbeg(C.nc); I < xend(C.nc); I += xstride()) {
    int X[3];
    unflat(C.n, I, X);
    C.b[I] = lv_restrict_one<Lv, R>(F, nd, X);
  }
}

// Prolongation fused with one post-smoothing sweep: y = x + xc[parent];
// xo = y + w (b - A y)/d (neighbour values of y formed on the fly).
template <typename Lv, typename R, bool OUT64>
__global__ void __launch_bounds__(TPB) k_v_post(Lv F, Lv C, int nd, R *__restrict__ xo, R omega,
                                                double *__restrict__ z, const double *__restrict__ dsc,
                                                const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  for (unsigned id = xbeg(F.nc); id < xend(F.nc); id += xstride()) {
    int c[3];
    unflat(F.n, id, c);
    const R y = F.x[id] + C.x[parent_of<R>(F.n, C.n, nd, c)];
    const R dg = F.diag[id];
    R ay = dg * y;
    for_neighbours(F.n, nd, id, c, [&](unsigned nid, int k) {
      int cn[3] = {c[0], c[1], c[2]};
      const int d = k >> 1;
      cn[d] += (k & 1) ? 1 : -1;
      const R yn = F.x[nid] + C.x[parent_of<R>(F.n, C.n, nd, cn)];
      ay += lv_off(F, id, c, k) * yn;
    });
    const R v = y + omega * (F.b[id] - ay) / dg;
    xo[id] = v;
    if (OUT64) z[id] = unscale((double)v, dsc, id);
  }
}

// ------------------------------------------------------------------ single-block coarse tail

template <typename Lv>
struct LevelPack {
  Lv lv[VC_MAX_LEVELS];
};

template <typename Lv, typename R>
__device__ void blk_jacobi(const Lv &L, int nd, const R *x, R *xo, R omega, bool zero_x)
{
  for (unsigned id = threadIdx.x; id < L.nc; id += blockDim.x) {
    if (zero_x) { xo[id] = omega * L.b[id] / L.diag[id]; continue; }
    int c[3];
    unflat(L.n, id, c);
    xo[id] = x[id] + omega * (L.b[id] - lv_apply(L, nd, x, id, c)) / L.diag[id];
  }
  __syncthreads();
}

// All levels l0..L-1 of a V-cycle in one block of VC_COARSE_TPB threads.  On
// entry lv[l0].b holds the right-hand side; on exit lv[l0].x holds the
// correction.  The coarsest level uses its dense inverse when it has at most
// 64 cells, else 64 damped-Jacobi sweeps.
template <typename Lv, typename R>
__global__ void __launch_bounds__(VC_COARSE_TPB) k_v_coarse_cycle(LevelPack<Lv> P, int l0, int L, int nd, int nu,
                                                                  R omega, const double *__restrict__ Ainv,
                                                                  const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  // bit l set: level l's current iterate lives in its t buffer
  unsigned par = 0;
#define VC_X(l) (((par >> (l)) & 1u) ? P.lv[l].t : P.lv[l].x)
#define VC_T(l) (((par >> (l)) & 1u) ? P.lv[l].x : P.lv[l].t)
  for (int l = l0; l < L - 1; ++l) {
    Lv F = P.lv[l];
    blk_jacobi<Lv, R>(F, nd, nullptr, VC_X(l), omega, true);
    for (int k = 1; k < nu; ++k) {
      blk_jacobi<Lv, R>(F, nd, VC_X(l), VC_T(l), omega, false);
      par ^= 1u << l;
    }
    F.x = VC_X(l);
    const Lv C = P.lv[l + 1];
    for (unsigned I = threadIdx.x; I < C.nc; I += blockDim.x) {
      int X[3];
      unflat(C.n, I, X);
      C.b[I] = lv_restrict_one<Lv, R>(F, nd, X);
    }
    __syncthreads();
  }
  {
    const Lv C = P.lv[L - 1];
    if (C.nc <= 64u) {
      R *xc = VC_X(L - 1);
      for (unsigned i = threadIdx.x; i < C.nc; i += blockDim.x) {
        double acc = 0.0;
        for (unsigned j = 0; j < C.nc; ++j) acc += Ainv[i * C.nc + j] * (double)C.b[j];
        xc[i] = (R)acc;
      }
      __syncthreads();
    } else {
      blk_jacobi<Lv, R>(C, nd, nullptr, VC_X(L - 1), omega, true);
      for (int k = 1; k < 64; ++k) {
        blk_jacobi<Lv, R>(C, nd, VC_X(L - 1), VC_T(L - 1), omega, false);
        par ^= 1u << (L - 1);
      }
    }
  }
  for (int l = L - 2; l >= l0; --l) {
    const Lv F = P.lv[l];
    const Lv C = P.lv[l + 1];
    R *xf = VC_X(l);
    const R *xc = VC_X(l + 1);
    for (unsigned id = threadIdx.x; id < F.nc; id += blockDim.x) {
      int c[3];
      unflat(F.n, id, c);
      xf[id] += xc[parent_of<R>(F.n, C.n, nd, c)];
    }
    __syncthreads();
    for (int k = 0; k < nu; ++k) {
      blk_jacobi<Lv, R>(F, nd, VC_X(l), VC_T(l), omega, false);
      par ^= 1u << l;
    }
  }
  // leave the result of level l0 in its x buffer
  if ((par >> l0) & 1u) {
    for (unsigned id = threadIdx.x; id < P.lv[l0].nc; id += blockDim.x) P.lv[l0].x[id] = P.lv[l0].t[id];
  }
#undef VC_X
#undef VC_T
}

// b = (R) r (level-0 input when the whole cycle runs in the single block).
template <typename Lv, typename R>
__global__ void __launch_bounds__(TPB) k_v_cast_in(Lv L, const double *__restrict__ r, const double *__restrict__ dsc,
                                                   double rscale, const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  for (unsigned id = xbeg(L.nc); id < xend(L.nc); id += xstride())
    L.b[id] = (R)(rscale * (dsc ? r[id] / sqrt(dsc[id]) : r[id]));
}

// z = (double) x
template <typename Lv, typename R>
__global__ void __launch_bounds__(TPB) k_v_cast_out(Lv L, double *__restrict__ z, const double *__restrict__ dsc,
                                                    const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  for (unsigned id = xbeg(L.nc); id < xend(L.nc); id += xstride()) z[id] = unscale((double)L.x[id], dsc, id);
}

}  // namespace vos
