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

// levels at or below this size run in the single-block kernel (3-D): a 16^3
// level costs the block more than its own multi-block launches do
constexpr int VC_BLOCK_MAX = 2048;
constexpr int VC_TAIL_2D = 2048;     // the same in 2-D (the tail runs in LDS, k_v_coarse_lds)
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
  return smg_off(L, k, id);
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

// Coarse right-hand side: the fine residual summed over each aggregate
// (children in cz, cy, cx order; a missing child -- ceil aggregation or an
// extent-1 dimension -- is evaluated at a clamped cell and skipped by a
// select, so no load sits in a branch).
template <typename Lv, typename R>
__device__ __forceinline__ R lv_restrict_one(const Lv &F, int nd, const int X[3])
{
  R s = 0;
  const int lz = nd == 3 ? 2 : 1;
#pragma unroll
  for (int cz = 0; cz < lz; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
        const int c0 = F.n[0] == 1 ? 0 : 2 * X[0] + cx, c1 = F.n[1] == 1 ? 0 : 2 * X[1] + cy;
        const int c2 = (nd == 3 && F.n[2] > 1) ? 2 * X[2] + cz : 0;
        const bool ok = !((F.n[0] == 1 && cx) || (F.n[1] == 1 && cy) || (cz && !(nd == 3 && F.n[2] > 1))) &&
                        c0 < F.n[0] && c1 < F.n[1] && c2 < F.n[2];
        const int c[3] = {min(c0, F.n[0] - 1), min(c1, F.n[1] - 1), min(c2, F.n[2] - 1)};
        const unsigned id = (unsigned)c[0] + (unsigned)F.n[0] * ((unsigned)c[1] + (unsigned)F.n[1] * (unsigned)c[2]);
        const R r = F.b[id] - lv_apply(F, nd, F.x, id, c);
        s = ok ? s + r : s;
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

// ------------------------------------------------------------------ 2-D tiled fine-level kernels
//
// On a 2-D level the launches of a fine level (pre-smoothing sweeps,
// restriction, prolongation + post-smoothing sweeps) become two: each block
// owns a VT_X x TY tile and recomputes the NU sweeps on a halo that shrinks
// by one cell per sweep (tile + NU, ..., tile + 1, tile), so no grid-wide
// synchronisation is needed between the sweeps.  Grid: tile_of().  Every cell value is formed by
// the same expression, in the same order, as in the unfused kernels above
// (sweeps 1-2 as k_v_pre, later pre-sweeps and the residual as k_v_jacobi /
// k_v_restrict, the first post-sweep as k_v_post, later ones as k_v_jacobi).

// Tiles are VT_X wide and TY high (both even: aggregates stay inside): TY =
// VT_Y_BIG on levels of at least VT_BIG_CELLS cells, where the larger tile
// halves the halo overhead, VT_Y_SMALL below, where more, smaller blocks
// shorten the latency-bound legs (micromodel step: 2.00 ms with 16
// everywhere, 1.88 ms with 4 and 1.97 ms with 2 everywhere, 1.87 ms with
// 16 / 4 and 1.83 ms with 16 / 2).
constexpr int VT_X = 32, VT_Y_BIG = 16, VT_Y_SMALL = 2;
constexpr unsigned VT_BIG_CELLS = 1u << 18;

// XCD-aware tile order: blocks are dispatched round-robin over the 8 XCDs
// (block b on XCD b % 8), so block b takes tile (b % 8) * per + b / 8 -- each
// XCD sweeps one contiguous band of tiles, and a tile's halo neighbours are
// mostly in the same XCD's L2.  Launch per * 8 blocks, per = ceil(tiles / 8).
template <int TY>
__device__ __forceinline__ bool tile_of(int nx, int ny, int &tx, int &ty)
{
  const int gx = (nx + VT_X - 1) / VT_X, gy = (ny + TY - 1) / TY;
  const unsigned ntiles = (unsigned)gx * (unsigned)gy;
  const unsigned per = (ntiles + NXCD - 1) / NXCD;
  const unsigned t = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  if (t >= ntiles) return false;
  tx = (int)(t % (unsigned)gx);
  ty = (int)(t / (unsigned)gx);
  return true;
}

template <int NU, int TY>
struct VHalo {
  static constexpr int W = VT_X + 2 * NU, H = TY + 2 * NU;
};

// Neighbour term from an LDS coefficient: SLevel adds off * x, MgLevel
// subtracts T * x (o = -T), matching lv_term.
template <typename R>
__device__ __forceinline__ R lds_term(const SLevel<R> &, R v, R o, R xn) { return v + o * xn; }
template <typename R>
__device__ __forceinline__ R lds_term(const MgLevel<R> &, R v, R o, R xn) { return v - (-o) * xn; }

// A x at a tile cell (lv_apply order) from the iterate x in LDS and the
// cell's own coefficients o[k] (towards neighbour slot k, 0 where there is
// no neighbour) and diagonal dg, held in registers by the thread that owns
// the cell.
template <typename Lv, typename R, int W>
__device__ __forceinline__ R tile_apply(const Lv &L, const R o[4], R dg, const R (*x)[W], int lx, int ly,
                                        const int c[3])
{
  R v = dg * x[ly][lx];
  if (c[0] > 0) v = lds_term(L, v, o[0], x[ly][lx - 1]);
  if (c[0] < L.n[0] - 1) v = lds_term(L, v, o[1], x[ly][lx + 1]);
  if (c[1] > 0) v = lds_term(L, v, o[2], x[ly - 1][lx]);
  if (c[1] < L.n[1] - 1) v = lds_term(L, v, o[3], x[ly + 1][lx]);
  return v;
}

// A x in the k_v_pre / k_v_post order: d x + sum of off * x.
template <typename Lv, typename R, int W>
__device__ __forceinline__ R tile_apply_off(const Lv &L, const R o[4], R dg, const R (*x)[W], int lx, int ly,
                                            const int c[3])
{
  R v = dg * x[ly][lx];
  if (c[0] > 0) v += o[0] * x[ly][lx - 1];
  if (c[0] < L.n[0] - 1) v += o[1] * x[ly][lx + 1];
  if (c[1] > 0) v += o[2] * x[ly - 1][lx];
  if (c[1] < L.n[1] - 1) v += o[3] * x[ly + 1][lx];
  return v;
}

// Cells of a staged tile-plus-halo that one thread owns for the whole
// kernel: cell t = threadIdx.x + i TPB of the W x H array (i < PER), with its
// right-hand side, diagonal and neighbour coefficients in registers.  Only
// the iterates (which neighbours read) live in LDS, so a block needs two W x H
// planes of LDS instead of eight and more blocks fit on a CU.
template <typename R, int W, int H>
struct TileCells {
  static constexpr int PER = (W * H + TPB - 1) / TPB;
  int lx[PER], ly[PER], gx[PER], gy[PER];
  bool in[PER];   // inside the level (and inside the staged array)
  R b[PER], d[PER], o[PER][4];
};

// Stage the owned cells of the tile whose LDS cell (0, 0) is level cell (X0,
// Y0): every load first (coordinates clamped into the level, so no load sits
// in a branch), then the values (defaults outside the level: b 0, diagonal 1,
// no coefficients).
template <typename Lv, typename R, int W, int H, bool FROM64>
__device__ __forceinline__ void tile_stage(const Lv &F, int X0, int Y0, const double *__restrict__ r64,
                                           const double *__restrict__ dsc, double rscale,
                                           TileCells<R, W, H> &T)
{
  constexpr int PER = TileCells<R, W, H>::PER;
  const int nx = F.n[0], ny = F.n[1];
  R rb[PER], rd[PER], ro[PER][4];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int t = min((int)threadIdx.x + i * TPB, W * H - 1);
    const int gx = min(max(X0 + t % W, 0), nx - 1), gy = min(max(Y0 + t / W, 0), ny - 1);
    const unsigned id = (unsigned)gx + (unsigned)nx * (unsigned)gy;
    const int c[3] = {gx, gy, 0};
    if (FROM64) rb[i] = (R)(rscale * (dsc ? r64[id] / sqrt(dsc[id]) : r64[id]));
    else rb[i] = F.b[id];
    rd[i] = F.diag[id];
#pragma unroll
    for (int k = 0; k < 4; ++k) ro[i][k] = lv_off(F, id, c, k);
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int t = (int)threadIdx.x + i * TPB;
    T.lx[i] = t % W;
    T.ly[i] = t / W;
    T.gx[i] = X0 + T.lx[i];
    T.gy[i] = Y0 + T.ly[i];
    const bool in = t < W * H && T.gx[i] >= 0 && T.gx[i] < nx && T.gy[i] >= 0 && T.gy[i] < ny;
    T.in[i] = in;
    T.b[i] = in ? rb[i] : (R)0;
    T.d[i] = in ? rd[i] : (R)1;
    T.o[i][0] = in && T.gx[i] > 0 ? ro[i][0] : (R)0;
    T.o[i][1] = in && T.gx[i] < nx - 1 ? ro[i][1] : (R)0;
    T.o[i][2] = in && T.gy[i] > 0 ? ro[i][2] : (R)0;
    T.o[i][3] = in && T.gy[i] < ny - 1 ? ro[i][3] : (R)0;
  }
}

// Owned cell i lies in the tile grown by h cells (the LDS array holds the tile
// grown by NU).
template <int NU, int TY, typename TC>
__device__ __forceinline__ bool tile_within(const TC &T, int i, int h)
{
  return T.in[i] && T.lx[i] >= NU - h && T.lx[i] < NU + VT_X + h && T.ly[i] >= NU - h && T.ly[i] < NU + TY + h;
}

// Down leg of a 2-D fine level: NU damped-Jacobi sweeps from zero, then the
// residual restricted to the coarse right-hand side.  F.x receives the
// smoothed iterate (tile cells); with FROM64, F.b the scaled right-hand side.
// Grid: tile_of(), block TPB.
template <typename Lv, typename R, bool FROM64, int NU, int TY>
__global__ void __launch_bounds__(TPB) k_v_down2d(Lv F, Lv C, const double *__restrict__ r64,
                                                  const double *__restrict__ dsc, double rscale, R omega,
                                                  const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  constexpr int W = VHalo<NU, TY>::W, H = VHalo<NU, TY>::H;
  __shared__ R xa[H][W], xb[H][W];
  const int nx = F.n[0], ny = F.n[1];
  int tx, ty;
  if (!tile_of<TY>(nx, ny, tx, ty)) return;
  const int X0 = tx * VT_X - NU, Y0 = ty * TY - NU;   // global coords of LDS cell (0, 0)
  TileCells<R, W, H> T;
  tile_stage<Lv, R, W, H, FROM64>(F, X0, Y0, r64, dsc, rscale, T);
  constexpr int PER = TileCells<R, W, H>::PER;
  // sweep 1 from zero on the whole staged array
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if ((int)threadIdx.x + i * TPB >= W * H) continue;
    if (FROM64 && T.in[i] && tile_within<NU, TY>(T, i, 0))
      F.b[(unsigned)T.gx[i] + (unsigned)nx * (unsigned)T.gy[i]] = T.b[i];
    xa[T.ly[i]][T.lx[i]] = T.in[i] ? omega * T.b[i] / T.d[i] : (R)0;
  }
  __syncthreads();
  // sweeps 2..NU on a halo shrinking from NU - 1 to 1 (ping-pong xa -> xb -> xa ...)
#pragma unroll
  for (int k = 2; k <= NU; ++k) {
    const int h = NU - k + 1;
    R(*src)[W] = (k % 2 == 0) ? xa : xb;
    R(*dst)[W] = (k % 2 == 0) ? xb : xa;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (!tile_within<NU, TY>(T, i, h)) continue;
      const int c[3] = {T.gx[i], T.gy[i], 0};
      const int lx = T.lx[i], ly = T.ly[i];
      const R ax = (k == 2) ? tile_apply_off<Lv, R, W>(F, T.o[i], T.d[i], src, lx, ly, c)
                            : tile_apply<Lv, R, W>(F, T.o[i], T.d[i], src, lx, ly, c);
      dst[ly][lx] = src[ly][lx] + omega * (T.b[i] - ax) / T.d[i];
    }
    __syncthreads();
  }
  R(*xf)[W] = (NU % 2 == 0) ? xb : xa;   // the last sweep's output
  R(*rs)[W] = (NU % 2 == 0) ? xa : xb;   // free now: the tile's residuals
  // residual on the tile, x to F.x
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    if (!tile_within<NU, TY>(T, i, 0)) continue;
    const int c[3] = {T.gx[i], T.gy[i], 0};
    const int lx = T.lx[i], ly = T.ly[i];
    F.x[(unsigned)T.gx[i] + (unsigned)nx * (unsigned)T.gy[i]] = xf[ly][lx];
    rs[ly][lx] = T.b[i] - tile_apply<Lv, R, W>(F, T.o[i], T.d[i], xf, lx, ly, c);
  }
  __syncthreads();
  // restriction: sum over each 2 x 2 aggregate (cy outer, cx inner); the tile
  // cells outside the level contribute nothing
  for (int t = threadIdx.x; t < (VT_X / 2) * (TY / 2); t += TPB) {
    const int ix = t % (VT_X / 2), iy = t / (VT_X / 2);
    const int IX = tx * (VT_X / 2) + ix, IY = ty * (TY / 2) + iy;
    if (IX >= C.n[0] || IY >= C.n[1]) continue;
    R sum = 0;
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) {
        if (2 * IX + cx >= nx || 2 * IY + cy >= ny) continue;
        sum += rs[NU + 2 * iy + cy][NU + 2 * ix + cx];
      }
    C.b[(unsigned)IX + (unsigned)C.n[0] * (unsigned)IY] = sum;
  }
}

// Up leg of a 2-D fine level: prolongation of the coarse correction and NU
// post-smoothing sweeps.  Reads F.x, F.b, C.x; writes the result to xo (a
// buffer other than F.x: neighbouring tiles still read F.x) and, with OUT64,
// z = unscale(result).
template <typename Lv, typename R, bool OUT64, int NU, int TY>
__global__ void __launch_bounds__(TPB) k_v_up2d(Lv F, Lv C, R *__restrict__ xo, R omega, double *__restrict__ z,
                                                const double *__restrict__ dsc, const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  constexpr int W = VHalo<NU, TY>::W, H = VHalo<NU, TY>::H;
  __shared__ R ya[H][W], yb[H][W];
  const int nx = F.n[0], ny = F.n[1];
  int tx, ty;
  if (!tile_of<TY>(nx, ny, tx, ty)) return;
  const int X0 = tx * VT_X - NU, Y0 = ty * TY - NU;
  constexpr int PER = TileCells<R, W, H>::PER;
  // the prolonged iterate, loaded with the other staging loads
  R rv[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int t = min((int)threadIdx.x + i * TPB, W * H - 1);
    const int gx = min(max(X0 + t % W, 0), nx - 1), gy = min(max(Y0 + t / W, 0), ny - 1);
    const int c[3] = {gx, gy, 0};
    rv[i] = F.x[(unsigned)gx + (unsigned)nx * (unsigned)gy] + C.x[parent_of<R>(F.n, C.n, 2, c)];
  }
  TileCells<R, W, H> T;
  tile_stage<Lv, R, W, H, false>(F, X0, Y0, nullptr, nullptr, 1.0, T);
#pragma unroll
  for (int i = 0; i < PER; ++i)
    if ((int)threadIdx.x + i * TPB < W * H) ya[T.ly[i]][T.lx[i]] = T.in[i] ? rv[i] : (R)0;
  __syncthreads();
#pragma unroll
  for (int k = 1; k <= NU; ++k) {
    const int h = NU - k;
    R(*src)[W] = (k % 2 == 1) ? ya : yb;
    R(*dst)[W] = (k % 2 == 1) ? yb : ya;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      if (!tile_within<NU, TY>(T, i, h)) continue;
      const int c[3] = {T.gx[i], T.gy[i], 0};
      const int lx = T.lx[i], ly = T.ly[i];
      const R ay = (k == 1) ? tile_apply_off<Lv, R, W>(F, T.o[i], T.d[i], src, lx, ly, c)
                            : tile_apply<Lv, R, W>(F, T.o[i], T.d[i], src, lx, ly, c);
      const R o = src[ly][lx] + omega * (T.b[i] - ay) / T.d[i];
      if (k < NU) {
        dst[ly][lx] = o;
      } else {
        const unsigned id = (unsigned)T.gx[i] + (unsigned)nx * (unsigned)T.gy[i];
        xo[id] = o;
        if (OUT64) z[id] = unscale((double)o, dsc, id);
      }
    }
    if (k < NU) __syncthreads();
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

// ------------------------------------------------------------------ 2-D coarse tail in LDS
//
// The same cycle as k_v_coarse_cycle for a 2-D tail whose first level has at
// most C0 x VC_COARSE_TPB cells and every later level at most VC_COARSE_TPB:
// thread i owns cells i + j VC_COARSE_TPB (j < C0) of the first level and cell
// i of the others, keeps their diagonals, neighbour coefficients and
// right-hand sides in registers, and the iterates live in LDS, so a sweep
// costs a barrier instead of a store and reload through L2.  Every value is
// formed by the expression k_v_coarse_cycle uses (bitwise equal results).
constexpr int VCL_MAXLV = 6;      // levels of the tail
constexpr int VCL_C0 = 4;         // most cells per thread on the first level
constexpr int VCL_CELLS = 5632;   // LDS cells over all levels of the tail

template <typename R>
struct CCoef {
  R d, o[4];   // diagonal; -x, +x, -y, +y coefficients as stored (MgLevel T, SLevel off)
};

template <typename R>
__device__ __forceinline__ CCoef<R> ccoef(const MgLevel<R> &L, unsigned id, const int c[3])
{
  const unsigned f0 = (unsigned)c[0] + (unsigned)L.fd[0][0] * ((unsigned)c[1] + (unsigned)L.fd[0][1] * c[2]);
  const unsigned f1 = (unsigned)c[0] + (unsigned)L.fd[1][0] * ((unsigned)c[1] + (unsigned)L.fd[1][1] * c[2]);
  return CCoef<R>{L.diag[id], {L.T[0][f0], L.T[0][f0 + 1], L.T[1][f1], L.T[1][f1 + L.fd[1][0]]}};
}

template <typename R>
__device__ __forceinline__ CCoef<R> ccoef(const SLevel<R> &L, unsigned id, const int *)
{
  return CCoef<R>{L.diag[id], {smg_off(L, 0, id), smg_off(L, 1, id), smg_off(L, 2, id), smg_off(L, 3, id)}};
}

template <typename R>
__device__ __forceinline__ R cterm(const MgLevel<R> &, R v, R o, R x) { return v - o * x; }
template <typename R>
__device__ __forceinline__ R cterm(const SLevel<R> &, R v, R o, R x) { return v + o * x; }

// A x at cell id of a 2-D level from the LDS iterate x (mg_apply_cell / smg_apply_cell order).
template <typename Lv, typename R>
__device__ __forceinline__ R capply(const Lv &L, const CCoef<R> &k, const R *x, unsigned id, const int c[3])
{
  const unsigned sy = (unsigned)L.n[0];
  const bool hw = c[0] > 0, he = c[0] < L.n[0] - 1, hs = c[1] > 0, hn = c[1] < L.n[1] - 1;
  const R xc = x[id], xw = x[hw ? id - 1 : id], xe = x[he ? id + 1 : id];
  const R xs = x[hs ? id - sy : id], xn = x[hn ? id + sy : id];
  R v = k.d * xc;
  v = hw ? cterm(L, v, k.o[0], xw) : v;
  v = he ? cterm(L, v, k.o[1], xe) : v;
  v = hs ? cterm(L, v, k.o[2], xs) : v;
  v = hn ? cterm(L, v, k.o[3], xn) : v;
  return v;
}

template <typename Lv, typename R, int C0>
__global__ void __launch_bounds__(VC_COARSE_TPB) k_v_coarse_lds(LevelPack<Lv> P, int l0, int L, int nu, R omega,
                                                                const double *__restrict__ Ainv,
                                                                const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  constexpr unsigned T = VC_COARSE_TPB;
  __shared__ R xs[2][VCL_CELLS];     // iterates (ping-pong), level q at offset off[q]
  __shared__ R rs[C0 * T];           // residuals being restricted; the coarsest right-hand side
  const int nl = L - l0;
  const unsigned i = threadIdx.x;
  unsigned off[VCL_MAXLV];
  CCoef<R> k[VCL_MAXLV][C0];
  R rb[VCL_MAXLV][C0];
  int sel[VCL_MAXLV];
  // slots of level q: C0 on the first level, 1 on the others
#define VCL_S(q) ((q) == 0 ? C0 : 1)
  {
    unsigned o = 0;
#pragma unroll
    for (int q = 0; q < VCL_MAXLV; ++q) {
      off[q] = o;
      sel[q] = 0;
#pragma unroll
      for (int j = 0; j < C0; ++j) {
        rb[q][j] = (R)0;
        k[q][j] = CCoef<R>{};
      }
      if (q < nl) {
        const Lv &F = P.lv[l0 + q];
        o += F.nc;
#pragma unroll
        for (int j = 0; j < VCL_S(q); ++j) {
          const unsigned id = i + j * T;
          if (id < F.nc) {
            int c[3];
            unflat(F.n, id, c);
            k[q][j] = ccoef(F, id, c);
            if (q == 0) rb[0][j] = F.b[id];
          }
        }
      }
    }
  }
  // Jacobi sweeps 2..count of level q (sweep 1, from zero, done before)
  auto sweeps = [&](int q, const Lv &F, int count) {
    for (int s = 1; s < count; ++s) {
      const R *xa = xs[sel[q]] + off[q];
      R *xb = xs[sel[q] ^ 1] + off[q];
#pragma unroll
      for (int j = 0; j < VCL_S(q); ++j) {
        const unsigned id = i + j * T;
        if (id < F.nc) {
          int c[3];
          unflat(F.n, id, c);
          xb[id] = xa[id] + omega * (rb[q][j] - capply(F, k[q][j], xa, id, c)) / k[q][j].d;
        }
      }
      sel[q] ^= 1;
      __syncthreads();
    }
  };
  auto zero_sweep = [&](int q, const Lv &F) {
#pragma unroll
    for (int j = 0; j < VCL_S(q); ++j) {
      const unsigned id = i + j * T;
      if (id < F.nc) xs[sel[q]][off[q] + id] = omega * rb[q][j] / k[q][j].d;
    }
    __syncthreads();
  };
#pragma unroll
  for (int q = 0; q < VCL_MAXLV - 1; ++q) {
    if (q < nl - 1) {
      const Lv &F = P.lv[l0 + q];
      zero_sweep(q, F);
      sweeps(q, F, nu);
#pragma unroll
      for (int j = 0; j < VCL_S(q); ++j) {
        const unsigned id = i + j * T;
        if (id < F.nc) {
          int c[3];
          unflat(F.n, id, c);
          rs[id] = rb[q][j] - capply(F, k[q][j], xs[sel[q]] + off[q], id, c);
        }
      }
      __syncthreads();
      // coarse right-hand side: the children's residuals in cy, cx order (lv_restrict_one)
      const Lv &C = P.lv[l0 + q + 1];
      if (i < C.nc) {
        int X[3];
        unflat(C.n, i, X);
        R sum = 0;
#pragma unroll
        for (int cy = 0; cy < 2; ++cy)
#pragma unroll
          for (int cx = 0; cx < 2; ++cx) {
            const int c0 = F.n[0] == 1 ? 0 : 2 * X[0] + cx, c1 = F.n[1] == 1 ? 0 : 2 * X[1] + cy;
            const bool ok = !((F.n[0] == 1 && cx) || (F.n[1] == 1 && cy)) && c0 < F.n[0] && c1 < F.n[1];
            const R r = rs[(unsigned)min(c0, F.n[0] - 1) + (unsigned)F.n[0] * (unsigned)min(c1, F.n[1] - 1)];
            sum = ok ? sum + r : sum;
          }
        rb[q + 1][0] = sum;
      }
      __syncthreads();
    }
  }
  // coarsest level (the first level too when the tail has one level)
#pragma unroll
  for (int q = 0; q < VCL_MAXLV; ++q) {
    if (q == nl - 1) {
      const Lv &C = P.lv[L - 1];
      if (C.nc <= 64u) {
        if (i < C.nc) rs[i] = rb[q][0];
        __syncthreads();
        if (i < C.nc) {
          double acc = 0.0;
          for (unsigned j = 0; j < C.nc; ++j) acc += Ainv[i * C.nc + j] * (double)rs[j];
          xs[0][off[q] + i] = (R)acc;
        }
        sel[q] = 0;
        __syncthreads();
      } else {
        zero_sweep(q, C);
        sweeps(q, C, 64);
      }
    }
  }
#pragma unroll
  for (int q = VCL_MAXLV - 2; q >= 0; --q) {
    if (q < nl - 1) {
      const Lv &F = P.lv[l0 + q];
      const Lv &C = P.lv[l0 + q + 1];
#pragma unroll
      for (int j = 0; j < VCL_S(q); ++j) {
        const unsigned id = i + j * T;
        if (id < F.nc) {
          int c[3];
          unflat(F.n, id, c);
          xs[sel[q]][off[q] + id] += xs[sel[q + 1]][off[q + 1] + parent_of<R>(F.n, C.n, 2, c)];
        }
      }
      __syncthreads();
      sweeps(q, F, nu + 1);
    }
  }
#pragma unroll
  for (int j = 0; j < C0; ++j) {
    const unsigned id = i + j * T;
    if (id < P.lv[l0].nc) P.lv[l0].x[id] = xs[sel[0]][off[0] + id];
  }
#undef VCL_S
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
