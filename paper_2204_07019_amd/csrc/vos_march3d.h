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
#include <algorithm>
#include <type_traits>

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

// Launch shapes (host side).
// z-run length of the marching kernels: about 2048 work
// items per level, even (restriction aggregates pairs of planes), 2..64.
inline int zrun_len(const int n[3])
{
  const long tiles = (long)((n[0] + ZT_X - 1) / ZT_X) * ((n[1] + ZT_Y - 1) / ZT_Y);
  long zl = (long)n[2] * tiles / 2048;
  zl = std::max(2L, std::min(64L, zl));
  return (int)(zl & ~1L);
}

// Blocks of a 3-D marching kernel: its work items rounded up to a multiple of the 8 XCDs.
inline unsigned zrun_blocks(const int n[3], int zlen)
{
  const unsigned nw = (unsigned)((n[0] + ZT_X - 1) / ZT_X) * (unsigned)((n[1] + ZT_Y - 1) / ZT_Y) *
                      (unsigned)((n[2] + zlen - 1) / zlen);
  return (nw + NXCD - 1) / NXCD * NXCD;
}

// The fused two-sweep legs (k_v_down3d / k_v_up3d) recompute a few planes at
// the start of every z-run and hold more LDS and registers per block than the
// separate kernels, so fewer blocks are resident per CU (slots = CUs x
// resident blocks per CU).  A launch then runs in rounds = ceil(blocks /
// slots) waves of resident blocks, each taking about (z-run + 3) plane times,
// so the runs are cut so that every block is resident at once, unless that
// leaves more than a quarter of the slots idle: then the run count is the one
// that minimises rounds x (z-run + 3) (384^3 with 144 FP64 tiles on 256
// slots: 7 runs of 56 planes in 4 rounds instead of one 384-plane run on 144
// CUs).  Runs are even and at least 8 planes long.  They run on levels of at least 2^20
// cells (the smaller levels keep the separate kernels).  Their tiles are
// ZT_X x zf_rows<R> cells for a level of R values, one thread per cell: 16
// rows for FP64 levels (fewer halo cells per tile cell; one 1024-thread block
// per CU), 8 for FP32 ones (three 512-thread blocks per CU fit their registers
// and LDS, which their latency-bound marches need more than a smaller halo).
template <typename R>
constexpr int zf_rows = sizeof(R) == 8 ? 16 : 8;
inline long zfused_tiles(const int n[3], int fy) { return (long)((n[0] + ZT_X - 1) / ZT_X) * ((n[1] + fy - 1) / fy); }
inline int zrun_len_fused(const int n[3], int slots, int fy)
{
  const long tiles = zfused_tiles(n, fy), sl = std::max(1, slots);
  const long runs0 = std::max(1L, sl / tiles);
  long z0 = ((long)n[2] + runs0 - 1) / runs0;
  z0 = std::max(8L, z0 + (z0 & 1));
  if (4 * tiles * (((long)n[2] + z0 - 1) / z0) >= 3 * sl) return (int)z0;
  long best = z0, best_cost = -1;
  for (long runs = 1; runs <= n[2]; ++runs) {
    long zl = ((long)n[2] + runs - 1) / runs;
    zl = std::max(8L, zl + (zl & 1));
    const long blocks = tiles * (((long)n[2] + zl - 1) / zl);
    const long cost = (blocks + sl - 1) / sl * (zl + 3);
    if (best_cost < 0 || cost < best_cost) {
      best_cost = cost;
      best = zl;
    }
  }
  return (int)best;
}
// Blocks of a fused-leg launch: its work items rounded up to a multiple of the 8 XCDs.
inline unsigned zrun_blocks_fused(const int n[3], int zlen, int fy)
{
  const unsigned nw = (unsigned)zfused_tiles(n, fy) * (unsigned)((n[2] + zlen - 1) / zlen);
  return (nw + NXCD - 1) / NXCD * NXCD;
}
inline bool zfused_level(const int n[3])
{
  return (unsigned long)n[0] * (unsigned long)n[1] * (unsigned long)n[2] >= (1ul << 20);
}

// The pressure operator marches through z on 3-D grids at least half a tile
// wide whose tiles fit the MAXB partial slots; the z-run is lengthened until
// the work items do.
inline bool papply_marching(const Dev &g)
{
  const long tiles = (long)((g.n[0] + ZT_X - 1) / ZT_X) * ((g.n[1] + ZT_Y - 1) / ZT_Y);
  return g.nd == 3 && g.n[0] >= ZT_X / 2 && g.n[1] >= 2 && g.n[2] >= 2 && tiles <= MAXB;
}

inline int papply_zlen(const Dev &g)
{
  const long tiles = (long)((g.n[0] + ZT_X - 1) / ZT_X) * ((g.n[1] + ZT_Y - 1) / ZT_Y);
  int zl = zrun_len(g.n);
  while (tiles * ((g.n[2] + zl - 1) / zl) > MAXB) zl += 2;
  return zl;
}

// One LDS plane: tile + one-cell halo, [y][x].
template <typename R>
using ZPlane = R[ZT_Y + 2][ZT_X + 2];

// Neighbour values of the thread's own cell: x/y from the LDS plane, z from registers.
template <typename R>
struct ZNb {
  R w, e, s, n, b, t;
};

// Diagonal and the six neighbour coefficients of a cell as stored (MgLevel:
// face transmissibilities T, subtracted; SLevel: off-diagonals, added), in
// the neighbour slot order -x, +x, -y, +y, -z, +z.  Loaded unconditionally
// (every index is inside its array) so that all loads of a plane are in
// flight together; a missing neighbour's term is skipped by a select.
template <typename R>
struct ZCoef {
  R d, o[6];
};

template <typename R>
__device__ __forceinline__ ZCoef<R> zcoef(const MgLevel<R> &L, unsigned id, const int c[3])
{
  ZCoef<R> k;
  const unsigned f0 = (unsigned)c[0] + (unsigned)L.fd[0][0] * ((unsigned)c[1] + (unsigned)L.fd[0][1] * c[2]);
  const unsigned f1 = (unsigned)c[0] + (unsigned)L.fd[1][0] * ((unsigned)c[1] + (unsigned)L.fd[1][1] * c[2]);
  const unsigned f2 = (unsigned)c[0] + (unsigned)L.fd[2][0] * ((unsigned)c[1] + (unsigned)L.fd[2][1] * c[2]);
  const unsigned sz = (unsigned)L.n[0] * L.n[1];
  k.o[0] = L.T[0][f0];
  k.o[1] = L.T[0][f0 + 1];
  k.o[2] = L.T[1][f1];
  k.o[3] = L.T[1][f1 + L.fd[1][0]];
  k.o[4] = L.T[2][f2];
  k.o[5] = L.T[2][f2 + sz];
  // finest level: the diagonal from the six faces by k_mg_diag's expression
  // (bitwise the stored value) instead of one more array read
  if (L.dsum) k.d = (k.o[0] + k.o[1] + k.o[2] + k.o[3]) + (k.o[4] + k.o[5]);
  else k.d = L.diag[id];
  return k;
}

template <typename R>
__device__ __forceinline__ ZCoef<R> zcoef(const SLevel<R> &L, unsigned id, const int *)
{
  ZCoef<R> k;
  k.d = L.diag[id];
#pragma unroll
  for (int q = 0; q < 6; ++q) k.o[q] = smg_off(L, q, id);
  return k;
}

// As zcoef, with the cell's stored diagonal dg already loaded by the caller.
template <typename R>
__device__ __forceinline__ ZCoef<R> zcoef_dg(const MgLevel<R> &L, unsigned, const int c[3], R dg)
{
  ZCoef<R> k;
  const unsigned f0 = (unsigned)c[0] + (unsigned)L.fd[0][0] * ((unsigned)c[1] + (unsigned)L.fd[0][1] * c[2]);
  const unsigned f1 = (unsigned)c[0] + (unsigned)L.fd[1][0] * ((unsigned)c[1] + (unsigned)L.fd[1][1] * c[2]);
  const unsigned f2 = (unsigned)c[0] + (unsigned)L.fd[2][0] * ((unsigned)c[1] + (unsigned)L.fd[2][1] * c[2]);
  const unsigned sz = (unsigned)L.n[0] * L.n[1];
  k.o[0] = L.T[0][f0];
  k.o[1] = L.T[0][f0 + 1];
  k.o[2] = L.T[1][f1];
  k.o[3] = L.T[1][f1 + L.fd[1][0]];
  k.o[4] = L.T[2][f2];
  k.o[5] = L.T[2][f2 + sz];
  k.d = L.dsum ? (k.o[0] + k.o[1] + k.o[2] + k.o[3]) + (k.o[4] + k.o[5]) : dg;
  return k;
}

template <typename R>
__device__ __forceinline__ ZCoef<R> zcoef_dg(const SLevel<R> &L, unsigned id, const int *, R dg)
{
  ZCoef<R> k;
  k.d = dg;
#pragma unroll
  for (int q = 0; q < 6; ++q) k.o[q] = smg_off(L, q, id);
  return k;
}

// The fused legs' coefficient loads: the level's own words (the FP32 copies
// of an SLevel are loaded by the legs' FP32 variant itself, as raw words).
template <typename R>
__device__ __forceinline__ ZCoef<R> zcoef_own(const MgLevel<R> &L, unsigned id, const int c[3])
{
  return zcoef(L, id, c);
}
template <typename R>
__device__ __forceinline__ ZCoef<R> zcoef_own(const SLevel<R> &L, unsigned id, const int *)
{
  ZCoef<R> k;
  k.d = L.diag[id];
#pragma unroll
  for (int q = 0; q < 6; ++q) k.o[q] = L.off[(size_t)q * L.nc + id];
  return k;
}
template <typename R>
__device__ __forceinline__ ZCoef<R> zcoef_own_dg(const MgLevel<R> &L, unsigned id, const int c[3], R dg)
{
  return zcoef_dg(L, id, c, dg);
}
template <typename R>
__device__ __forceinline__ ZCoef<R> zcoef_own_dg(const SLevel<R> &L, unsigned id, const int *, R dg)
{
  ZCoef<R> k;
  k.d = dg;
#pragma unroll
  for (int q = 0; q < 6; ++q) k.o[q] = L.off[(size_t)q * L.nc + id];
  return k;
}
// FP32 off-diagonal copies of an SLevel as loaded (O32 variant of the fused legs).
template <typename Lv>
__device__ __forceinline__ void zoff32_load(const Lv &, unsigned, float (&)[6])
{
}
template <typename R>
__device__ __forceinline__ void zoff32_load(const SLevel<R> &L, unsigned id, float (&o)[6])
{
#pragma unroll
  for (int q = 0; q < 6; ++q) o[q] = L.off32[(size_t)q * L.nc + id];
}

// Which neighbour slots exist.
struct ZHas {
  bool h[6];
};
__device__ __forceinline__ ZHas zhas(const int n[3], const int c[3])
{
  return ZHas{{c[0] > 0, c[0] < n[0] - 1, c[1] > 0, c[1] < n[1] - 1, c[2] > 0, c[2] < n[2] - 1}};
}

template <typename R>
__device__ __forceinline__ R zterm(const MgLevel<R> &, R v, R o, R x) { return v - o * x; }
template <typename R>
__device__ __forceinline__ R zterm(const SLevel<R> &, R v, R o, R x) { return v + o * x; }

// A x in the lv_apply order (mg_apply_cell / smg_apply_cell).
template <typename Lv, typename R>
__device__ __forceinline__ R zapply(const Lv &L, const ZHas &h, const ZCoef<R> &k, R xc, const ZNb<R> &x)
{
  R v = k.d * xc;
  v = h.h[0] ? zterm(L, v, k.o[0], x.w) : v;
  v = h.h[1] ? zterm(L, v, k.o[1], x.e) : v;
  v = h.h[2] ? zterm(L, v, k.o[2], x.s) : v;
  v = h.h[3] ? zterm(L, v, k.o[3], x.n) : v;
  v = h.h[4] ? zterm(L, v, k.o[4], x.b) : v;
  v = h.h[5] ? zterm(L, v, k.o[5], x.t) : v;
  return v;
}

// Neighbour coefficient as lv_off gives it: -T (MgLevel) or off (SLevel).
template <typename R>
__device__ __forceinline__ R zoff(const MgLevel<R> &, R o) { return -o; }
template <typename R>
__device__ __forceinline__ R zoff(const SLevel<R> &, R o) { return o; }

// A x in the k_v_pre / k_v_post order: d x + lv_off * x over the neighbour slots.
template <typename Lv, typename R>
__device__ __forceinline__ R zapply_off(const Lv &L, const ZHas &h, const ZCoef<R> &k, R dg, R xc, const ZNb<R> &x)
{
  R v = dg * xc;
  v = h.h[0] ? v + zoff(L, k.o[0]) * x.w : v;
  v = h.h[1] ? v + zoff(L, k.o[1]) * x.e : v;
  v = h.h[2] ? v + zoff(L, k.o[2]) * x.s : v;
  v = h.h[3] ? v + zoff(L, k.o[3]) * x.n : v;
  v = h.h[4] ? v + zoff(L, k.o[4]) * x.b : v;
  v = h.h[5] ? v + zoff(L, k.o[5]) * x.t : v;
  return v;
}

// The march.  O: per-cell record whose member s is the staged value; K: the
// per-cell data the body reads (coefficients, right-hand side).
//   own(id, c)  -> O   the thread's own cell
//   halo(id, c) -> R   the staged value of a halo cell
//   coef(id, c) -> K   loaded before the plane's barrier
//   body(in, id, c, cur, nb, k)  plane z of the own cell, called by every
//                     thread of the block (in == false outside the level) so
//                     that body may hold block-uniform barriers
// own and halo are called for every thread with an in-range cell (the level's
// cell 0 when the thread has none) and their result is discarded there, so
// that their loads are not split into branches.
template <typename R, typename O, typename K, typename OwnF, typename HaloF, typename CoefF, typename BodyF>
__device__ __forceinline__ void zmarch(const int n[3], const ZTile &t, ZPlane<R> *pl, OwnF own, HaloF halo,
                                       CoefF coef, BodyF body)
{
  __shared__ R dump[TPB];   // halo stores of threads without a halo cell (never read)
  const int nx = n[0], ny = n[1], nz = n[2];
  const unsigned sz = (unsigned)nx * (unsigned)ny;
  const int lx = threadIdx.x % ZT_X, ly = threadIdx.x / ZT_X;
  const int gx = t.x0 + lx, gy = t.y0 + ly;
  const bool in = gx < nx && gy < ny;
  const unsigned col = in ? (unsigned)gx + (unsigned)nx * (unsigned)gy : 0u;   // column of cell (0, 0) outside
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

  auto own_at = [&](int z) -> O {
    const bool ok = in && z >= 0 && z < nz;
    const int c[3] = {ok ? gx : 0, ok ? gy : 0, ok ? z : 0};
    const O o = own(ok ? col + sz * (unsigned)z : 0u, c);
    return ok ? o : O{};
  };
  auto halo_at = [&](int z, bool want) -> R {
    const bool ok = want && hin && z < nz;
    const int c[3] = {ok ? hgx : 0, ok ? hgy : 0, ok ? z : 0};
    const R v = halo(ok ? hcol + sz * (unsigned)z : 0u, c);
    return ok ? v : (R)0;
  };

  // LDS slot of this thread's halo value in each plane (a private dump slot without one)
  auto hslot = [&](int slot) -> R * { return hx >= 0 ? &pl[slot][hy][hx] : &dump[threadIdx.x]; };

  R sm = t.z0 > 0 ? own_at(t.z0 - 1).s : (R)0;   // own staged value of plane z - 1
  O cur = own_at(t.z0);
  {
    const R hv = halo_at(t.z0, true);
    pl[0][ly + 1][lx + 1] = cur.s;
    *hslot(0) = hv;
  }
  int s = 0;
  for (int z = t.z0; z < t.z1; ++z) {
    const int s1 = s == 2 ? 0 : s + 1;
    const int c[3] = {gx, gy, z};
    const unsigned id = col + sz * (unsigned)z;
    // loads of plane z + 1's staged values and of plane z's coefficients, all
    // unconditional (outside the level: cell (0, 0, z), result unused)
    const O nxt = own_at(z + 1);
    const R hv = halo_at(z + 1, z + 1 < t.z1);
    const int cs[3] = {in ? gx : 0, in ? gy : 0, z};
    const K k = coef(id, cs);
    pl[s1][ly + 1][lx + 1] = nxt.s;
    *hslot(s1) = hv;
    __syncthreads();
    const ZPlane<R> &p = pl[s];
    ZNb<R> nb;
    nb.w = p[ly + 1][lx];
    nb.e = p[ly + 1][lx + 2];
    nb.s = p[ly][lx + 1];
    nb.n = p[ly + 2][lx + 1];
    nb.b = sm;
    nb.t = nxt.s;
    body(in, id, c, cur, nb, k);
    sm = cur.s;
    cur = nxt;
    s = s1;
  }
}

// Coefficients and right-hand side of a cell.
template <typename R>
struct ZCoefB {
  ZCoef<R> a;
  R b;
};

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
  zmarch<R, O, ZCoefB<R>>(
      L.n, t, pl, [&](unsigned id, const int *) { return O{x[id]}; }, [&](unsigned id, const int *) { return x[id]; },
      [&](unsigned id, const int *c) { return ZCoefB<R>{zcoef(L, id, c), L.b[id]}; },
      [&](bool in, unsigned id, const int c[3], const O &cur, const ZNb<R> &nb, const ZCoefB<R> &k) {
        if (!in) return;
        const R v = cur.s + omega * (k.b - zapply(L, zhas(L.n, c), k.a, cur.s, nb)) / k.a.d;
        // the cycle's last sweep: only its output z is read afterwards
        if (OUT64) z[id] = unscale((double)v, dsc, id);
        else xo[id] = v;
      });
}

// Right-hand side of a pre-smoothing kernel: the level's b (RHS_B), or on
// level 0 the FP64 residual (R)(rscale r) (RHS_R) or (R)(rscale r / sqrt(dsc))
// (RHS_RD) -- k_v_pre's FROM64 expression with the dsc test taken on the host
// -- or, in the fused legs only, the FP64 vector r times the level's own
// diagonal, (R)(r d) (RHS_RG: the cycle's input formed where the diagonal is
// already loaded; the product is rounded on its own, never contracted into a
// later fused multiply-add, so it is bitwise the vector r d that the caller
// would otherwise store).
enum { RHS_B = 0, RHS_R = 1, RHS_RD = 2, RHS_RG = 3 };


// Pre-smoothing sweeps 1 and 2 (k_v_pre with two sweeps).
template <typename Lv, typename R, int RHS>
__global__ void __launch_bounds__(TPB) k_v_pre3d(Lv L, const double *__restrict__ r64,
                                                 const double *__restrict__ dsc, double rscale, R omega, int zlen,
                                                 const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  ZTile t;
  if (!ztile_of(L.n, zlen, t)) return;
  __shared__ ZPlane<R> pl[3];
  struct O { R s, bb, dg; };
  constexpr bool FROM64 = RHS != RHS_B;
  auto rhs = [&](unsigned id) -> R {
    if (RHS == RHS_RD) return (R)(rscale * (r64[id] / sqrt(dsc[id])));
    if (RHS == RHS_R) return (R)(rscale * r64[id]);
    return L.b[id];
  };
  zmarch<R, O, ZCoef<R>>(
      L.n, t, pl,
      [&](unsigned id, const int *) {
        O o;
        o.bb = rhs(id);
        o.dg = L.diag[id];
        o.s = omega * o.bb / o.dg;
        return o;
      },
      [&](unsigned id, const int *) { return omega * rhs(id) / L.diag[id]; },
      [&](unsigned id, const int *c) { return zcoef(L, id, c); },
      [&](bool in, unsigned id, const int c[3], const O &cur, const ZNb<R> &nb, const ZCoef<R> &k) {
        if (!in) return;
        if (FROM64) L.b[id] = cur.bb;
        const R ax = zapply_off<Lv, R>(L, zhas(L.n, c), k, cur.dg, cur.s, nb);
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
  zmarch<R, O, ZCoefB<R>>(
      F.n, t, pl, [&](unsigned id, const int *) { return O{x[id]}; }, [&](unsigned id, const int *) { return x[id]; },
      [&](unsigned id, const int *c) { return ZCoefB<R>{zcoef(F, id, c), F.b[id]}; },
      [&](bool in, unsigned id, const int c[3], const O &cur, const ZNb<R> &nb, const ZCoefB<R> &k) {
        const int z = c[2];
        rs[z & 1][ly][lx] = in ? k.b - zapply(F, zhas(F.n, c), k.a, cur.s, nb) : (R)0;
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
  zmarch<R, O, ZCoefB<R>>(
      F.n, t, pl, [&](unsigned id, const int *c) { return O{yv(id, c)}; }, yv,
      [&](unsigned id, const int *c) { return ZCoefB<R>{zcoef(F, id, c), F.b[id]}; },
      [&](bool in, unsigned id, const int c[3], const O &cur, const ZNb<R> &nb, const ZCoefB<R> &k) {
        if (!in) return;
        const R dg = k.a.d;
        const R ay = zapply_off<Lv, R>(F, zhas(F.n, c), k.a, dg, cur.s, nb);
        const R v = cur.s + omega * (k.b - ay) / dg;
        if (OUT64) z[id] = unscale((double)v, dsc, id);
        else xo[id] = v;
      });
}

// ---------------------------------------------------------------------------
// Fused finest-level legs of a V-cycle with two sweeps each way.  The separate
// kernels above read the level's coefficients four times per cycle (two
// pre-sweeps, restriction, prolongation + first up sweep, second up sweep).
// Here one march does two stencil passes: stage 0 forms a pointwise value v on
// the tile plus a two-cell x/y halo (plane z + 2), stage 1 applies the first
// stencil to v on the tile plus a one-cell halo (plane z + 1), stage 2 applies
// the second stencil on the tile itself (plane z).  The halo cells' stage-1
// values are recomputed by both blocks that need them, so each tile cell's
// coefficients cross HBM about once per leg.  Every value is formed by the
// expression of the separate kernel it replaces (k_v_pre3d + k_v_restrict3d
// down, k_v_post3d + k_v_jacobi3d up), so the cycle's results are bitwise
// those of the separate kernels.
//
// Tiles are ZT_X x FY cells (FY = zf_rows<R>) with one thread per cell: the
// first halo ring carries 2 (ZT_X + 2 + FY) cells, 29 % of a 64 x 8 tile's
// cells, 16 % of a 64 x 16 one's (55 % with 4 rows).  LDS: four v planes
// (two-cell halo; a plane is read by three consecutive stage-1 passes, so
// four slots let stage 0 run one plane ahead with one barrier per plane) and
// two u planes (one-cell halo).  A thread owns its tile cell (stages 0-2), at
// most one cell of the one-cell ring (stages 0-1) and at most one of the
// two-cell ring (stage 0).
constexpr int ZH2_X = ZT_X + 4;   // two-cell halo plane width
constexpr int ZH1_X = ZT_X + 2;   // one-cell halo plane width
template <int FY>
struct ZFS {   // the shape of an FY-row fused tile
  static constexpr int TPB = ZT_X * FY;
  static constexpr int H2Y = FY + 4, H1Y = FY + 2;   // halo plane heights
  static constexpr int RING1 = 2 * ZH1_X + 2 * FY, RING2 = 2 * ZH2_X + 2 * (FY + 2);
  static_assert(RING1 <= TPB && RING2 <= TPB, "one ring cell per thread");
  static_assert(FY % 2 == 0, "restriction aggregates stay inside a tile");
};

// Work item of a fused-leg block: as ztile_of, with ZT_X x FY tiles.
template <int FY>
__device__ __forceinline__ bool zftile_of(const int n[3], int zlen, ZTile &t)
{
  const unsigned gx = (unsigned)(n[0] + ZT_X - 1) / ZT_X, gy = (unsigned)(n[1] + FY - 1) / FY;
  const unsigned gz = (unsigned)(n[2] + zlen - 1) / (unsigned)zlen;
  const unsigned tiles = gx * gy, nw = tiles * gz;
  const unsigned per = (nw + NXCD - 1) / NXCD;
  const unsigned w = (blockIdx.x % NXCD) * per + blockIdx.x / NXCD;
  if (w >= nw) return false;
  const unsigned zr = w / tiles, tt = w - zr * tiles;
  t.x0 = (int)(tt % gx) * ZT_X;
  t.y0 = (int)(tt / gx) * FY;
  t.z0 = (int)zr * zlen;
  t.z1 = min(n[2], t.z0 + zlen);
  return true;
}

// Position (in two-halo plane coordinates) of the thread's cell of class k:
// 0 its tile cell, 1 its one-cell-ring cell, 2 its two-cell-ring cell;
// false when the thread has none.
template <int FY>
__device__ __forceinline__ bool zfused_cell(int k, int &hx, int &hy)
{
  using S = ZFS<FY>;
  const int h = threadIdx.x;
  if (k == 0) {
    hx = h % ZT_X + 2;
    hy = h / ZT_X + 2;
    return true;
  }
  if (k == 1) {
    if (h >= S::RING1) return false;
    int x1, y1;   // one-halo coordinates
    if (h < ZH1_X) { x1 = h; y1 = 0; }
    else if (h < 2 * ZH1_X) { x1 = h - ZH1_X; y1 = S::H1Y - 1; }
    else if (h < 2 * ZH1_X + FY) { x1 = 0; y1 = h - 2 * ZH1_X + 1; }
    else { x1 = ZH1_X - 1; y1 = h - 2 * ZH1_X - FY + 1; }
    hx = x1 + 1;
    hy = y1 + 1;
    return true;
  }
  if (h >= S::RING2) return false;
  if (h < ZH2_X) { hx = h; hy = 0; }
  else if (h < 2 * ZH2_X) { hx = h - ZH2_X; hy = S::H2Y - 1; }
  else if (h < 2 * ZH2_X + FY + 2) { hx = 0; hy = h - 2 * ZH2_X + 1; }
  else { hx = ZH2_X - 1; hy = h - 2 * ZH2_X - (FY + 2) + 1; }
  return true;
}

// A cell of the march: its two-halo plane position, level coordinates and column.
struct ZCell {
  int hx, hy, gx, gy;
  bool has, in;     // the thread has this cell; it lies inside the level (x, y)
  unsigned col;     // gx + nx gy (0 outside)
};

template <int FY>
__device__ __forceinline__ ZCell zfused_at(int k, const ZTile &t, const int n[3])
{
  ZCell c;
  c.has = zfused_cell<FY>(k, c.hx, c.hy);
  if (!c.has) { c.hx = c.hy = 2; }   // a position whose neighbours are in the plane (never stored)
  c.gx = t.x0 + c.hx - 2;
  c.gy = t.y0 + c.hy - 2;
  c.in = c.has && c.gx >= 0 && c.gx < n[0] && c.gy >= 0 && c.gy < n[1];
  c.col = c.in ? (unsigned)c.gx + (unsigned)n[0] * (unsigned)c.gy : 0u;
  return c;
}

// In-plane neighbours of two-halo position (hx, hy) from a two-halo plane,
// z neighbours from the planes below and above.
template <typename R>
__device__ __forceinline__ ZNb<R> znb2(const R (*pl)[ZH2_X], const R (*lo)[ZH2_X], const R (*hi)[ZH2_X], int hx,
                                       int hy)
{
  ZNb<R> nb;
  nb.w = pl[hy][hx - 1];
  nb.e = pl[hy][hx + 1];
  nb.s = pl[hy - 1][hx];
  nb.n = pl[hy + 1][hx];
  nb.b = lo[hy][hx];
  nb.t = hi[hy][hx];
  return nb;
}

// Down leg: the two pre-smoothing sweeps of k_v_pre3d (from the FP64 residual,
// RHS_R, or the level's b, RHS_B) and the residual restriction of
// k_v_restrict3d, in one march.  Writes x (after the second sweep) and the
// coarse b.  With RHS_R the level's b is not stored: the finest level's up leg
// forms it again from the same residual by the same expression.  O32: the
// level's off-diagonals are read from its FP32 copies, carried as loaded and
// widened after the plane's barrier.  zlen even.
template <typename Lv, typename R, int RHS, bool O32>
__global__ void __launch_bounds__(ZT_X * zf_rows<R>) k_v_down3d(Lv F, Lv C, const double *__restrict__ r64, double rscale,
                                                              R omega,
                                                  int zlen, const double *__restrict__ sc)
{
  static_assert(RHS == RHS_R || RHS == RHS_B || RHS == RHS_RG, "no dsc scaling in the fused leg");
  if (sc[S_CONV] != 0.0) return;
  ZTile t;
  constexpr int FY = zf_rows<R>, H2Y = ZFS<FY>::H2Y;
  if (!zftile_of<FY>(F.n, zlen, t)) return;
  __shared__ R vpl[4][H2Y][ZH2_X];
  __shared__ R upl[2][H2Y][ZH2_X];   // one-halo values, kept in two-halo coordinates
  __shared__ R rs[2][FY][ZT_X];
  const int nz = F.n[2];
  const unsigned sz = (unsigned)F.n[0] * (unsigned)F.n[1];
  const ZCell c0 = zfused_at<FY>(0, t, F.n), c1 = zfused_at<FY>(1, t, F.n), c2 = zfused_at<FY>(2, t, F.n);
  // the right-hand side as loaded (the FP64 vector r or the level's b) and as
  // used with the cell's diagonal d, (R)(rscale r), (R)(r d) or b: loads carry
  // the raw word, so that no arithmetic ahead of a plane's barrier waits for them
  constexpr bool R64 = RHS == RHS_R || RHS == RHS_RG;
  using RB = typename std::conditional<R64, double, R>::type;
  auto rhs_raw = [&](unsigned id) -> RB {
    if constexpr (R64) return r64[id];
    else return F.b[id];
  };
  auto rhs = [&](RB raw, R d) -> R {
    if constexpr (RHS == RHS_R) return (R)(rscale * raw);
    else if constexpr (RHS == RHS_RG) return (R)mul_rounded(raw, (double)d);
    else return raw;
  };
  // stage 0: v = omega b / d (the first sweep from x = 0), 0 outside the level.
  // Its inputs for the thread's three cells are loaded one plane ahead (load0,
  // every index inside the arrays) and carried in registers to put0.
  const ZCell *cs[3] = {&c0, &c1, &c2};
  struct P0 { RB b[3]; R d[3]; };
  auto load0 = [&](int z) -> P0 {
    P0 p;
    const bool zin = z >= 0 && z < nz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const unsigned id = cs[k]->in && zin ? cs[k]->col + sz * (unsigned)z : 0u;
      p.b[k] = rhs_raw(id);
      p.d[k] = F.diag[id];
    }
    return p;
  };
  auto put0 = [&](int z, const P0 &p) {
    const int s = z & 3;
    const bool zin = z >= 0 && z < nz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R v = omega * rhs(p.b[k], p.d[k]) / p.d[k];
      if (cs[k]->has) vpl[s][cs[k]->hy][cs[k]->hx] = cs[k]->in && zin ? v : (R)0;
    }
  };
  // stage 1 for one cell at plane z: the second sweep (k_v_pre3d's expression);
  // its loads (load1) are issued before the plane's barrier, the arithmetic
  // (apply1) after it
  struct S1 { R u; RB bb; R dg; ZCoef<R> k; float k32[6]; };
  auto load1 = [&](const ZCell &c, int z) -> S1 {
    S1 o;
    const bool ok = c.in && z >= 0 && z < nz;
    const int cc[3] = {ok ? c.gx : 0, ok ? c.gy : 0, ok ? z : 0};
    const unsigned id = ok ? c.col + sz * (unsigned)z : 0u;
    o.bb = rhs_raw(id);
    o.dg = F.diag[id];
    if constexpr (O32) {
      o.k.d = o.dg;
      zoff32_load(F, id, o.k32);
    } else {
      o.k = zcoef_own(F, id, cc);
    }
    o.u = (R)0;
    return o;
  };
  // the same, with b and d of class-k cell c taken from stage 0's loads p of
  // that plane (the same words): only the off-diagonals are loaded
  auto load1p = [&](const ZCell &c, int z, const P0 &p, int k) -> S1 {
    S1 o;
    const bool ok = c.in && z >= 0 && z < nz;
    const int cc[3] = {ok ? c.gx : 0, ok ? c.gy : 0, ok ? z : 0};
    const unsigned id = ok ? c.col + sz * (unsigned)z : 0u;
    o.bb = p.b[k];
    o.dg = p.d[k];
    if constexpr (O32) {
      o.k.d = p.d[k];
      zoff32_load(F, id, o.k32);
    } else {
      o.k = zcoef_own_dg(F, id, cc, p.d[k]);
    }
    o.u = (R)0;
    return o;
  };
  auto apply1 = [&](const ZCell &c, int z, S1 &o) {
    if constexpr (O32) {
#pragma unroll
      for (int q = 0; q < 6; ++q) o.k.o[q] = (R)o.k32[q];
    }
    const bool ok = c.in && z >= 0 && z < nz;
    const int cc[3] = {ok ? c.gx : 0, ok ? c.gy : 0, ok ? z : 0};
    const R s = vpl[z & 3][c.hy][c.hx];
    const ZNb<R> nb = znb2<R>(vpl[z & 3], vpl[(z - 1) & 3], vpl[(z + 1) & 3], c.hx, c.hy);
    const R ax = zapply_off<Lv, R>(F, zhas(F.n, cc), o.k, o.dg, s, nb);
    o.u = ok ? s + omega * (rhs(o.bb, o.dg) - ax) / o.dg : (R)0;
  };
  auto stage1 = [&](const ZCell &c, int z) -> S1 {
    S1 o = load1(c, z);
    apply1(c, z, o);
    return o;
  };
  const int lx = threadIdx.x % ZT_X, ly = threadIdx.x / ZT_X;
  // prologue: v on planes z0-2 .. z0+1, u on planes z0-1 and z0; stage 0's
  // loads of plane z+1 (held) and z+2 (ahead) enter the march's plane z
  for (int z = t.z0 - 2; z <= t.z0; ++z) put0(z, load0(z));
  P0 held = load0(t.z0 + 1);
  put0(t.z0 + 1, held);
  P0 ahead = load0(t.z0 + 2);
  __syncthreads();
  R u_prev, u_cur;
  ZCoef<R> k_cur;
  R b_cur;
  {
    const S1 a = stage1(c0, t.z0 - 1);
    const S1 a1 = stage1(c1, t.z0 - 1);
    if (c1.has) upl[(t.z0 - 1) & 1][c1.hy][c1.hx] = a1.u;
    upl[(t.z0 - 1) & 1][c0.hy][c0.hx] = a.u;
    u_prev = a.u;
    const S1 b = stage1(c0, t.z0);
    const S1 b1 = stage1(c1, t.z0);
    if (c1.has) upl[t.z0 & 1][c1.hy][c1.hx] = b1.u;
    upl[t.z0 & 1][c0.hy][c0.hx] = b.u;
    u_cur = b.u;
    k_cur = b.k;
    b_cur = rhs(b.bb, b.dg);
    if (c0.in) F.x[c0.col + sz * (unsigned)t.z0] = b.u;
  }
  // one plane of the march, called twice per loop trip as in the up leg
  auto plane = [&](int z) {
    S1 a = load1p(c0, z + 1, held, 0), a1 = load1p(c1, z + 1, held, 1);
    const P0 next = load0(z + 3);
    put0(z + 2, ahead);
    held = ahead;
    ahead = next;
    __syncthreads();
    // stage 1 on plane z + 1
    apply1(c0, z + 1, a);
    apply1(c1, z + 1, a1);
    if (c1.has) upl[(z + 1) & 1][c1.hy][c1.hx] = a1.u;
    upl[(z + 1) & 1][c0.hy][c0.hx] = a.u;
    if (c0.in && z + 1 < t.z1) F.x[c0.col + sz * (unsigned)(z + 1)] = a.u;
    // stage 2 on plane z: the residual of the second sweep (k_v_restrict3d's expression)
    {
      const int cc[3] = {c0.gx, c0.gy, z};
      ZNb<R> nb;
      nb.w = upl[z & 1][c0.hy][c0.hx - 1];
      nb.e = upl[z & 1][c0.hy][c0.hx + 1];
      nb.s = upl[z & 1][c0.hy - 1][c0.hx];
      nb.n = upl[z & 1][c0.hy + 1][c0.hx];
      nb.b = u_prev;
      nb.t = a.u;
      rs[z & 1][ly][lx] = c0.in ? b_cur - zapply(F, zhas(F.n, cc), k_cur, u_cur, nb) : (R)0;
    }
    u_prev = u_cur;
    u_cur = a.u;
    k_cur = a.k;
    b_cur = rhs(a.bb, a.dg);
    if ((z & 1) == 0 && z + 1 < nz) return;   // block-uniform
    __syncthreads();
    if (threadIdx.x < (ZT_X / 2) * (FY / 2)) {
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
  };
  int z = t.z0;
  for (; z + 1 < t.z1; z += 2) {
    plane(z);
    plane(z + 1);
  }
  if (z < t.z1) plane(z);   // block-uniform
}

// Up leg: the prolongation with the first post-smoothing sweep of k_v_post3d
// and the second sweep of k_v_jacobi3d, in one march.  Writes the result to
// xo, or with OUT64 (the finest level: the cycle's last sweep) only to the
// FP64 output z; there the right-hand side is (R)(rscale r64), the down leg's
// expression, since that leg did not store it, or with RG (R)(r64 d), the
// RHS_RG expression with the cell's diagonal d.  O32 as in the down leg.
template <typename Lv, typename R, bool OUT64, bool O32, bool RG = false>
__global__ void __launch_bounds__(ZT_X * zf_rows<R>) k_v_up3d(Lv F, Lv C, R *__restrict__ xo, R omega,
                                                            double *__restrict__ z64,
                                                const double *__restrict__ dsc, const double *__restrict__ r64,
                                                double rscale, int zlen, const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  ZTile t;
  constexpr int FY = zf_rows<R>, H2Y = ZFS<FY>::H2Y;
  if (!zftile_of<FY>(F.n, zlen, t)) return;
  __shared__ R vpl[4][H2Y][ZH2_X];
  __shared__ R upl[2][H2Y][ZH2_X];
  const int nz = F.n[2];
  const unsigned sz = (unsigned)F.n[0] * (unsigned)F.n[1];
  const ZCell c0 = zfused_at<FY>(0, t, F.n), c1 = zfused_at<FY>(1, t, F.n), c2 = zfused_at<FY>(2, t, F.n);
  // stage 0: y = x + the coarse correction of the cell's aggregate; inputs
  // loaded one plane ahead as in the down leg
  const ZCell *cs[3] = {&c0, &c1, &c2};
  struct P0 { R x[3], e[3]; };
  auto load0 = [&](int z) -> P0 {
    P0 p;
    const bool zin = z >= 0 && z < nz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const bool ok = cs[k]->in && zin;
      const int cc[3] = {ok ? cs[k]->gx : 0, ok ? cs[k]->gy : 0, ok ? z : 0};
      const unsigned id = ok ? cs[k]->col + sz * (unsigned)z : 0u;
      p.x[k] = F.x[id];
      p.e[k] = C.x[parent_of<R>(F.n, C.n, 3, cc)];
    }
    return p;
  };
  auto put0 = [&](int z, const P0 &p) {
    const int s = z & 3;
    const bool zin = z >= 0 && z < nz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const R v = p.x[k] + p.e[k];
      if (cs[k]->has) vpl[s][cs[k]->hy][cs[k]->hx] = cs[k]->in && zin ? v : (R)0;
    }
  };
  // stage 1: the first up sweep (k_v_post3d's expression), loads before the
  // plane's barrier (load1), arithmetic after it (apply1); the right-hand side
  // is carried as loaded (the FP64 residual with OUT64) and formed at its use
  static_assert(OUT64 || !RG, "the diagonal-scaled input is the finest level's");
  using RB = typename std::conditional<OUT64, double, R>::type;
  auto rhs = [&](RB raw, R d) -> R {
    if constexpr (RG) return (R)mul_rounded(raw, (double)d);
    else if constexpr (OUT64) return (R)(rscale * raw);
    else return raw;
  };
  struct S1 { R u; ZCoef<R> k; RB b; float k32[6]; };
  auto load1 = [&](const ZCell &c, int z) -> S1 {
    S1 o;
    const bool ok = c.in && z >= 0 && z < nz;
    const int cc[3] = {ok ? c.gx : 0, ok ? c.gy : 0, ok ? z : 0};
    const unsigned id = ok ? c.col + sz * (unsigned)z : 0u;
    if constexpr (O32) {
      o.k.d = F.diag[id];
      zoff32_load(F, id, o.k32);
    } else {
      o.k = zcoef_own(F, id, cc);
    }
    if constexpr (OUT64) o.b = r64[id];
    else o.b = F.b[id];
    o.u = (R)0;
    return o;
  };
  auto apply1 = [&](const ZCell &c, int z, S1 &o) {
    if constexpr (O32) {
#pragma unroll
      for (int q = 0; q < 6; ++q) o.k.o[q] = (R)o.k32[q];
    }
    const bool ok = c.in && z >= 0 && z < nz;
    const int cc[3] = {ok ? c.gx : 0, ok ? c.gy : 0, ok ? z : 0};
    const R y = vpl[z & 3][c.hy][c.hx];
    const ZNb<R> nb = znb2<R>(vpl[z & 3], vpl[(z - 1) & 3], vpl[(z + 1) & 3], c.hx, c.hy);
    const R dg = o.k.d;
    const R ay = zapply_off<Lv, R>(F, zhas(F.n, cc), o.k, dg, y, nb);
    o.u = ok ? y + omega * (rhs(o.b, dg) - ay) / dg : (R)0;
  };
  auto stage1 = [&](const ZCell &c, int z) -> S1 {
    S1 o = load1(c, z);
    apply1(c, z, o);
    return o;
  };
  R u_prev, u_cur, b_cur;
  ZCoef<R> k_cur;
  for (int z = t.z0 - 2; z <= t.z0 + 1; ++z) put0(z, load0(z));
  P0 ahead = load0(t.z0 + 2);
  __syncthreads();
  {
    const S1 a = stage1(c0, t.z0 - 1);
    const S1 a1 = stage1(c1, t.z0 - 1);
    if (c1.has) upl[(t.z0 - 1) & 1][c1.hy][c1.hx] = a1.u;
    upl[(t.z0 - 1) & 1][c0.hy][c0.hx] = a.u;
    u_prev = a.u;
    const S1 b = stage1(c0, t.z0);
    const S1 b1 = stage1(c1, t.z0);
    if (c1.has) upl[t.z0 & 1][c1.hy][c1.hx] = b1.u;
    upl[t.z0 & 1][c0.hy][c0.hx] = b.u;
    u_cur = b.u;
    k_cur = b.k;
    b_cur = rhs(b.b, b.k.d);
  }
  // one plane of the march; called twice per loop trip (the compiler does not
  // unroll a loop with a barrier itself), which saves some of the copies of the
  // values carried from plane to plane
  auto plane = [&](int z) {
    S1 a = load1(c0, z + 1), a1 = load1(c1, z + 1);
    const P0 next = load0(z + 3);
    put0(z + 2, ahead);
    ahead = next;
    __syncthreads();
    apply1(c0, z + 1, a);
    apply1(c1, z + 1, a1);
    if (c1.has) upl[(z + 1) & 1][c1.hy][c1.hx] = a1.u;
    upl[(z + 1) & 1][c0.hy][c0.hx] = a.u;
    // stage 2 on plane z: the second sweep (k_v_jacobi3d's expression)
    if (c0.in) {
      const int cc[3] = {c0.gx, c0.gy, z};
      const unsigned id = c0.col + sz * (unsigned)z;
      ZNb<R> nb;
      nb.w = upl[z & 1][c0.hy][c0.hx - 1];
      nb.e = upl[z & 1][c0.hy][c0.hx + 1];
      nb.s = upl[z & 1][c0.hy - 1][c0.hx];
      nb.n = upl[z & 1][c0.hy + 1][c0.hx];
      nb.b = u_prev;
      nb.t = a.u;
      const R v = u_cur + omega * (b_cur - zapply(F, zhas(F.n, cc), k_cur, u_cur, nb)) / k_cur.d;
      if (OUT64) z64[id] = unscale((double)v, dsc, id);
      else xo[id] = v;
    }
    u_prev = u_cur;
    u_cur = a.u;
    k_cur = a.k;
    b_cur = rhs(a.b, a.k.d);
  };
  int z = t.z0;
  for (; z + 1 < t.z1; z += 2) {
    plane(z);
    plane(z + 1);
  }
  if (z < t.z1) plane(z);   // block-uniform
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
    struct K { double tw, te, ts, tn, tb, tt; };
    zmarch<double, O, K>(
        g.n, t, pl, [&](unsigned id, const int *) { return O{p[id]}; },
        [&](unsigned id, const int *) { return p[id]; },
        [&](unsigned, const int *c) {
          const unsigned f0 = fidx(g, 0, c[0], c[1], c[2]);
          const unsigned f1 = fidx(g, 1, c[0], c[1], c[2]);
          const unsigned f2 = fidx(g, 2, c[0], c[1], c[2]);
          const unsigned sy = (unsigned)g.fd[1][0], sz = (unsigned)g.n[0] * g.n[1];
          const K k{T0[f0], T0[f0 + 1], T1[f1], T1[f1 + sy], T2[f2], T2[f2 + sz]};
          // keep the loads ahead of the plane's barrier (one memory round trip per plane)
          asm volatile("" ::"v"(k.tw), "v"(k.te), "v"(k.ts), "v"(k.tn), "v"(k.tb), "v"(k.tt));
          return k;
        },
        [&](bool in, unsigned id, const int c[3], const O &cur, const ZNb<double> &nb, const K &k) {
          if (!in) return;
          const ZHas h = zhas(g.n, c);
          const double pc = cur.s;
          double v = (k.tw + k.te) * pc;
          v = h.h[0] ? v - k.tw * nb.w : v;
          v = h.h[1] ? v - k.te * nb.e : v;
          v += (k.ts + k.tn) * pc;
          v = h.h[2] ? v - k.ts * nb.s : v;
          v = h.h[3] ? v - k.tn * nb.n : v;
          v += (k.tb + k.tt) * pc;
          v = h.h[4] ? v - k.tb * nb.b : v;
          v = h.h[5] ? v - k.tt * nb.t : v;
          q[id] = v;
          acc += pc * v;
        });
  }
  const double vv[1] = {acc};
  write_partials<1>(vv, part);
}

}  // namespace vos
