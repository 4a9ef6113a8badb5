// vos_march3d.h -- z-marching kernels on 3-D grids: the fine multigrid
// levels of every hierarchy and the pressure operator of the outer CG.
//
// The plain fine-level kernels of vos_vcycle.h evaluate the 7-point stencil
// of every cell with its six neighbours fetched through the caches.  On a
// 256^3 level the neighbour planes (power-of-two strides) and the y-halos of
// other blocks' rows do not survive in L2 and come again from the Infinity
// Cache / HBM: up to 3x the arrays' size per launch.  Here a block owns a
// ZT_X x ZT_Y column tile and walks through a run of zlen planes.  The value
// the neighbours need (x, the first sweep's x1 or the prolonged y) is formed
// once per cell and plane; the plane's tile plus a one-cell x/y halo goes
// through LDS (a ring of three planes, one barrier per plane), and each
// thread keeps its own cell's z-1 / z / z+1 values in registers.  Every cell
// value is formed by the same expression, in the same order, as in the plain
// kernel it stands for (k_v_pre, k_v_jacobi, k_v_restrict, k_v_post,
// k_p_apply), so the level results are bitwise identical; the pressure
// operator's p.q partials are summed in the march's order instead.
//
// Work items are (z-run, tile) pairs numbered z-run major; block b runs on
// XCD b % 8 and takes item (b % 8) * per + b / 8, so each XCD walks one slab
// of z-runs and the halos its tiles share stay in its L2.
#pragma once
#include "vos_vcycle.h"

namespace vos {

constexpr int ZT_X = 64, ZT_Y = 4;   // one wave64 per tile row; both even (aggregates stay inside)
static_assert(ZT_X * ZT_Y == TPB, "one cell per thread and plane");

struct ZTile {
  int x0, y0, z0, z1;
};

__device__ __forceinline__ bool ztile_of(const int n[3], int zlen, ZTile &t)
{
  const unsigned gx = (unsigned)(n[0] + ZT_X - 1) / ZT_X, gy = (unsigned)(n[1] + ZT_Y - 1) / ZT_Y;
  const unsigned gz = (unsigned)(n[2] + zlen - 1) / (unsigned)zlen;
  const unsigned tiles = gx * gy, nw = tiles * gz;
  const unsigned per = (nw + NXCD - 1) / NXCD;
  const unsigned w = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  if (w >= nw) return false;
  const unsigned zr = w / tiles, tt = w - zr * tiles;
  t.x0 = (int)(tt % gx) * ZT_X;
  t.y0 = (int)(tt / gx) * ZT_Y;
  t.z0 = (int)zr * zlen;
  t.z1 = min(n[2], t.z0 + zlen);
  return true;
}

// One LDS plane: tile + one-cell halo, [y][x].
template <typename R>
using ZPlane = R[ZT_Y + 2][ZT_X + 2];

// Neighbour values of the thread's own cell: x/y from the LDS plane, z from registers.
template <typename R>
struct ZNb {
  R w, e, s, n, b, t;
};

// A x in the lv_apply order (mg_apply_cell / smg_apply_cell) from explicit neighbour values.
template <typename R>
__device__ __forceinline__ R zapply(const MgLevel<R> &L, unsigned id, const int c[3], R xc, const ZNb<R> &x)
{
  const unsigned f0 = (unsigned)c[0] + (unsigned)L.fd[0][0] * ((unsigned)c[1] + (unsigned)L.fd[0][1] * c[2]);
  const R tw = L.T[0][f0], te = L.T[0][f0 + 1];
  R v = L.diag[id] * xc;
  if (c[0] > 0) v -= tw * x.w;
  if (c[0] < L.n[0] - 1) v -= te * x.e;
  const unsigned f1 = (unsigned)c[0] + (unsigned)L.fd[1][0] * ((unsigned)c[1] + (unsigned)L.fd[1][1] * c[2]);
  const R ts = L.T[1][f1], tn = L.T[1][f1 + L.fd[1][0]];
  if (c[1] > 0) v -= ts * x.s;
  if (c[1] < L.n[1] - 1) v -= tn * x.n;
  const unsigned sz = (unsigned)L.n[0] * L.n[1];
  const unsigned f2 = (unsigned)c[0] + (unsigned)L.fd[2][0] * ((unsigned)c[1] + (unsigned)L.fd[2][1] * c[2]);
  const R tb = L.T[2][f2], tt = L.T[2][f2 + sz];
  if (c[2] > 0) v -= tb * x.b;
  if (c[2] < L.n[2] - 1) v -= tt * x.t;
  return v;
}

template <typename R>
__device__ __forceinline__ R zapply(const SLevel<R> &L, unsigned id, const int c[3], R xc, const ZNb<R> &x)
{
  R v = L.diag[id] * xc;
  const unsigned nc = L.nc;
  if (c[0] > 0) v += L.off[id] * x.w;
  if (c[0] < L.n[0] - 1) v += L.off[nc + id] * x.e;
  if (c[1] > 0) v += L.off[2 * nc + id] * x.s;
  if (c[1] < L.n[1] - 1) v += L.off[3 * nc + id] * x.n;
  if (c[2] > 0) v += L.off[4 * nc + id] * x.b;
  if (c[2] < L.n[2] - 1) v += L.off[5 * nc + id] * x.t;
  return v;
}

// A x in the k_v_pre / k_v_post order: d x + lv_off * x over the neighbour slots.
template <typename Lv, typename R>
__device__ __forceinline__ R zapply_off(const Lv &L, unsigned id, const int c[3], R dg, R xc, const ZNb<R> &x)
{
  R v = dg * xc;
  if (c[0] > 0) v += lv_off(L, id, c, 0) * x.w;
  if (c[0] < L.n[0] - 1) v += lv_off(L, id, c, 1) * x.e;
  if (c[1] > 0) v += lv_off(L, id, c, 2) * x.s;
  if (c[1] < L.n[1] - 1) v += lv_off(L, id, c, 3) * x.n;
  if (c[2] > 0) v += lv_off(L, id, c, 4) * x.b;
  if (c[2] < L.n[2] - 1) v += lv_off(L, id, c, 5) * x.t;
  return v;
}

// The march.  O: per-cell record whose member s is the staged value.
//   own(id, c)  -> O   the thread's own cell (reads only)
//   halo(id, c) -> R   the staged value of a halo cell
//   body(in, id, c, cur, nb)  plane z of the own cell (called by every thread
//                     of the block, in == false outside the level, so that
//                     body may hold block-uniform barriers)
template <typename R, typename O, typename OwnF, typename HaloF, typename BodyF>
__device__ __forceinline__ void zmarch(const int n[3], const ZTile &t, ZPlane<R> *pl, OwnF own, HaloF halo,
                                       BodyF body)
{
  const int nx = n[0], ny = n[1], nz = n[2];
  const unsigned sz = (unsigned)nx * (unsigned)ny;
  const int lx = threadIdx.x % ZT_X, ly = threadIdx.x / ZT_X;
  const int gx = t.x0 + lx, gy = t.y0 + ly;
  const bool in = gx < nx && gy < ny;
  const unsigned col = in ? (unsigned)gx + (unsigned)nx * (unsigned)gy : 0u;
  // this thread's halo cell (136 of them: rows above and below, columns left and right)
  int hx = -1, hy = -1;
  {
    const int h = threadIdx.x;
    if (h < ZT_X) { hx = h + 1; hy = 0; }
    else if (h < 2 * ZT_X) { hx = h - ZT_X + 1; hy = ZT_Y + 1; }
    else if (h < 2 * ZT_X + ZT_Y) { hx = 0; hy = h - 2 * ZT_X + 1; }
    else if (h < 2 * ZT_X + 2 * ZT_Y) { hx = ZT_X + 1; hy = h - 2 * ZT_X - ZT_Y + 1; }
  }
  const int hgx = t.x0 + hx - 1, hgy = t.y0 + hy - 1;
  const bool hin = hx >= 0 && hgx >= 0 && hgx < nx && hgy >= 0 && hgy < ny;
  const unsigned hcol = hin ? (unsigned)hgx + (unsigned)nx * (unsigned)hgy : 0u;

  auto stage = [&](int z, int slot, bool with_halo, O &o) {
    o = O{};
    if (in && z < nz) {
      const int c[3] = {gx, gy, z};
      o = own(col + sz * (unsigned)z, c);
    }
    pl[slot][ly + 1][lx + 1] = o.s;
    if (with_halo && hx >= 0) {
      R v = (R)0;
      if (hin && z < nz) {
        const int c[3] = {hgx, hgy, z};
        v = halo(hcol + sz * (unsigned)z, c);
      }
      pl[slot][hy][hx] = v;
    }
  };

  R sm = (R)0;   // own staged value of plane z - 1
  if (t.z0 > 0 && in) {
    const int c[3] = {gx, gy, t.z0 - 1};
    sm = own(col + sz * (unsigned)(t.z0 - 1), c).s;
  }
  O cur, nxt;
  stage(t.z0, 0, true, cur);
  int s = 0;
  for (int z = t.z0; z < t.z1; ++z) {
    const int s1 = s == 2 ? 0 : s + 1;
    stage(z + 1, s1, z + 1 < t.z1, nxt);
    __syncthreads();
    const ZPlane<R> &p = pl[s];
    ZNb<R> nb;
    nb.w = p[ly + 1][lx];
    nb.e = p[ly + 1][lx + 2];
    nb.s = p[ly][lx + 1];
    nb.n = p[ly + 2][lx + 1];
    nb.b = sm;
    nb.t = nxt.s;
    const int c[3] = {gx, gy, z};
    body(in, col + sz * (unsigned)z, c, cur, nb);
    sm = cur.s;
    cur = nxt;
    s = s1;
  }
}

// One damped-Jacobi sweep (k_v_jacobi).
template <typename Lv, typename R, bool OUT64>
__global__ void __launch_bounds__(TPB) k_v_jacobi3d(Lv L, const R *__restrict__ x, R *__restrict__ xo, R omega,
                                                    double *__restrict__ z, const double *__restrict__ dsc, int zlen,
                                                    const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  ZTile t;
  if (!ztile_of(L.n, zlen, t)) return;
  __shared__ ZPlane<R> pl[3];
  struct O { R s; };
  zmarch<R, O>(
      L.n, t, pl, [&](unsigned id, const int *) { return O{x[id]}; }, [&](unsigned id, const int *) { return x[id]; },
      [&](bool in, unsigned id, const int c[3], const O &cur, const ZNb<R> &nb) {
        if (!in) return;
        const R v = cur.s + omega * (L.b[id] - zapply(L, id, c, cur.s, nb)) / L.diag[id];
        xo[id] = v;
        if (OUT64) z[id] = unscale((double)v, dsc, id);
      });
}

// Pre-smoothing sweeps 1 and 2 (k_v_pre with two sweeps).
template <typename Lv, typename R, bool FROM64>
__global__ void __launch_bounds__(TPB) k_v_pre3d(Lv L, const double *__restrict__ r64,
                                                 const double *__restrict__ dsc, double rscale, R omega, int zlen,
                                                 const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  ZTile t;
  if (!ztile_of(L.n, zlen, t)) return;
  __shared__ ZPlane<R> pl[3];
  struct O { R s, bb, dg; };
  auto rhs = [&](unsigned id) -> R {
    if (FROM64) return (R)(rscale * (dsc ? r64[id] / sqrt(dsc[id]) : r64[id]));
    return L.b[id];
  };
  zmarch<R, O>(
      L.n, t, pl,
      [&](unsigned id, const int *) {
        O o;
        o.bb = rhs(id);
        o.dg = L.diag[id];
        o.s = omega * o.bb / o.dg;
        return o;
      },
      [&](unsigned id, const int *) { return omega * rhs(id) / L.diag[id]; },
      [&](bool in, unsigned id, const int c[3], const O &cur, const ZNb<R> &nb) {
        if (!in) return;
        if (FROM64) L.b[id] = cur.bb;
        const R ax = zapply_off<Lv, R>(L, id, c, cur.dg, cur.s, nb);
        L.x[id] = cur.s + omega * (cur.bb - ax) / cur.dg;
      });
}

// Residual restricted to the coarse right-hand side (k_v_restrict).  zlen even.
template <typename Lv, typename R>
__global__ void __launch_bounds__(TPB) k_v_restrict3d(Lv F, Lv C, int zlen, const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  ZTile t;
  if (!ztile_of(F.n, zlen, t)) return;
  __shared__ ZPlane<R> pl[3];
  __shared__ R rs[2][ZT_Y][ZT_X];   // residuals of the two planes of an aggregate layer
  struct O { R s; };
  const R *x = F.x;
  const int lx = threadIdx.x % ZT_X, ly = threadIdx.x / ZT_X;
  zmarch<R, O>(
      F.n, t, pl, [&](unsigned id, const int *) { return O{x[id]}; }, [&](unsigned id, const int *) { return x[id]; },
      [&](bool in, unsigned id, const int c[3], const O &cur, const ZNb<R> &nb) {
        const int z = c[2];
        rs[z & 1][ly][lx] = in ? F.b[id] - zapply(F, id, c, cur.s, nb) : (R)0;
        if ((z & 1) == 0 && z + 1 < F.n[2]) return;   // block-uniform
        __syncthreads();
        // sum over each 2 x 2 x 2 aggregate (cz, cy, cx from outer to inner)
        if (threadIdx.x < (ZT_X / 2) * (ZT_Y / 2)) {
          const int ix = threadIdx.x % (ZT_X / 2), iy = threadIdx.x / (ZT_X / 2);
          const int IX = t.x0 / 2 + ix, IY = t.y0 / 2 + iy, IZ = z >> 1;
          if (IX < C.n[0] && IY < C.n[1]) {
            R sum = 0;
            for (int cz = 0; cz < 2; ++cz)
              for (int cy = 0; cy < 2; ++cy)
                for (int cx = 0; cx < 2; ++cx) {
                  if (2 * IX + cx >= F.n[0] || 2 * IY + cy >= F.n[1] || 2 * IZ + cz >= F.n[2]) continue;
                  sum += rs[cz][2 * iy + cy][2 * ix + cx];
                }
            C.b[(unsigned)IX + (unsigned)C.n[0] * ((unsigned)IY + (unsigned)C.n[1] * (unsigned)IZ)] = sum;
          }
        }
      });
}

// Prolongation fused with the first post-smoothing sweep (k_v_post).
template <typename Lv, typename R, bool OUT64>
__global__ void __launch_bounds__(TPB) k_v_post3d(Lv F, Lv C, R *__restrict__ xo, R omega, double *__restrict__ z,
                                                  const double *__restrict__ dsc, int zlen,
                                                  const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  ZTile t;
  if (!ztile_of(F.n, zlen, t)) return;
  __shared__ ZPlane<R> pl[3];
  struct O { R s; };
  auto yv = [&](unsigned id, const int *c) -> R { return F.x[id] + C.x[parent_of<R>(F.n, C.n, 3, c)]; };
  zmarch<R, O>(
      F.n, t, pl, [&](unsigned id, const int *c) { return O{yv(id, c)}; }, yv,
      [&](bool in, unsigned id, const int c[3], const O &cur, const ZNb<R> &nb) {
        if (!in) return;
        const R dg = F.diag[id];
        const R ay = zapply_off<Lv, R>(F, id, c, dg, cur.s, nb);
        const R v = cur.s + omega * (F.b[id] - ay) / dg;
        xo[id] = v;
        if (OUT64) z[id] = unscale((double)v, dsc, id);
      });
}

// Pressure operator q = A p in papply_cell's expression order, with the
// per-block partials of p.q (quantity 0).  Every launched block writes its
// partial (zero without a work item).
__global__ void __launch_bounds__(TPB) k_p_apply3d(Dev g, const double *__restrict__ T0,
                                                   const double *__restrict__ T1, const double *__restrict__ T2,
                                                   const double *__restrict__ p, double *__restrict__ q,
                                                   double *__restrict__ part, int zlen, const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  __shared__ ZPlane<double> pl[3];
  double acc = 0.0;
  ZTile t;
  if (ztile_of(g.n, zlen, t)) {
    struct O { double s; };
    zmarch<double, O>(
        g.n, t, pl, [&](unsigned id, const int *) { return O{p[id]}; },
        [&](unsigned id, const int *) { return p[id]; },
        [&](bool in, unsigned id, const int c[3], const O &cur, const ZNb<double> &nb) {
          if (!in) return;
          const double pc = cur.s;
          const unsigned f0 = fidx(g, 0, c[0], c[1], c[2]);
          const double tw = T0[f0], te = T0[f0 + 1];
          double v = (tw + te) * pc;
          if (c[0] > 0) v -= tw * nb.w;
          if (c[0] < g.n[0] - 1) v -= te * nb.e;
          const unsigned f1 = fidx(g, 1, c[0], c[1], c[2]);
          const unsigned sy = (unsigned)g.fd[1][0];
          const double ts = T1[f1], tn = T1[f1 + sy];
          v += (ts + tn) * pc;
          if (c[1] > 0) v -= ts * nb.s;
          if (c[1] < g.n[1] - 1) v -= tn * nb.n;
          const unsigned f2 = fidx(g, 2, c[0], c[1], c[2]);
          const unsigned sz = (unsigned)g.n[0] * g.n[1];
          const double tb = T2[f2], tt = T2[f2 + sz];
          v += (tb + tt) * pc;
          if (c[2] > 0) v -= tb * nb.b;
          if (c[2] < g.n[2] - 1) v -= tt * nb.t;
          q[id] = v;
          acc += pc * v;
        });
  }
  const double vv[1] = {acc};
  write_partials<1>(vv, part);
}

}  // namespace vos
