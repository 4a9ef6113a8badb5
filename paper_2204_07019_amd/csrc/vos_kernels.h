// vos_kernels.h -- gfx950 kernels of one Volume-of-Solid step (coefficients,
// momentum predictor, pressure equation, correction, transport, reaction).
//
// All kernels are grid-stride sweeps of TPB threads over one cell or face
// grid; they are bandwidth-bound (well under 1 FLOP per byte), so the design
// goal is one coalesced pass per array and reductions fused into the sweep
// that produces their operands (wave64 shuffles + one LDS stage, partial sums
// per block, summed in fixed order by a one-block kernel: deterministic).
#pragma once
#include "vos_device.h"

namespace vos {

// Solver scalar block (device memory, one per Krylov solve).
enum Scal {
  S_RZ = 0, S_ALPHA, S_BETA, S_BN2, S_RES2, S_TOL2, S_CONV, S_ITS, S_PQ, S_ZQ,
  S_RHO, S_OMEGA, S_SHALF, S_BAD,
  S_RES0,          // squared residual norm at the solve's start (the SIMPLE loop's convergence test)
  S_TRUE,          // squared norm of the true residual b - A x at a converged BiCGStab iterate
  S_COUNT = 16
};

// ---------------------------------------------------------------- S1

// Momentum-unknown classification of the Laplacian neighbour of face (D, x)
// in direction e, side s: 0 unknown, 1 fixed face (value from *fv),
// 2 mirrored no-slip ghost, 3 zero-gradient ghost.
template <int D>
__device__ __forceinline__ int mom_nb(const Dev &g, const int x[3], int e, int s, double u_in, double *fv)
{
  *fv = 0.0;
  const int y = x[e] + s;
  if (e == D) {
    if (D == 0) {
      if (y == 0 && !g.drive) { *fv = u_in; return 1; }
      if (y > g.n[0] || y < 0) return 3;
      return 0;
    }
    if (y == 0 || y == g.n[D]) return 1;
    return 0;
  }
  if (y >= 0 && y < g.n[e]) return 0;
  if (e == 0) return y < 0 ? 2 : 3;
  return 2;
}

template <int D>
__device__ __forceinline__ bool mom_unknown(const Dev &g, const int x[3])
{
  const int q = x[D];
  return (q > 0 && q < g.n[D]) || (D == 0 && (q == g.n[0] || (q == 0 && g.drive)));
}

// eps on face (D, x): mean of the two cells inside, the adjacent cell on a boundary.
template <int D>
__device__ __forceinline__ double face_eps(const Dev &g, const double *eps, const int x[3], unsigned *lo, unsigned *hi)
{
  const unsigned c = cidx(g, x[0] < g.n[0] ? x[0] : g.n[0] - 1, x[1] < g.n[1] ? x[1] : g.n[1] - 1,
                          x[2] < g.n[2] ? x[2] : g.n[2] - 1);
  const unsigned st = D == 0 ? 1u : (D == 1 ? (unsigned)g.n[0] : (unsigned)g.n[0] * g.n[1]);
  const int q = x[D];
  if (q > 0 && q < g.n[D]) { *lo = c - st; *hi = c; return 0.5 * (eps[c - st] + eps[c]); }
  if (q == 0) { *lo = c; *hi = c; return eps[c]; }
  *lo = c; *hi = c;  // q == n[D]: c is the last cell (clamped above)
  return eps[c];
}

// Face coefficients of direction D: eps_f-scaled momentum diagonal dmom,
// pressure-correction coefficient af = rho/(eps_f dt) + beta_f and
// transmissibility T = S / (af d_f) (d_f = dx/2 on the outlet and, under the
// pressure drive, the inlet).  SIMPLE: steady momentum diagonal a / relax_u
// (no inertia) and the pressure correction of SIMPLE, af = dmom / eps_f.
template <int D>
__global__ void __launch_bounds__(TPB) k_face_coef(Dev g, Phys P, double dt, const double *__restrict__ eps,
                                                   double *__restrict__ dmom, double *__restrict__ af,
                                                   double *__restrict__ T)
{
  const double cvis = P.mu / (g.dx * g.dx);
  for (unsigned f = xbeg(g.nf[D]); f < xend(g.nf[D]); f += xstride()) {
    int x[3];
    unflat(g.fd[D], f, x);
    if (!mom_unknown<D>(g, x)) { dmom[f] = 1.0; af[f] = 0.0; T[f] = 0.0; continue; }
    unsigned lo, hi;
    const double ef = face_eps<D>(g, eps, x, &lo, &hi);
    const double om = 1.0 - ef;
    const double beta = P.mu * om * om / (P.k0 * ef * ef * ef);   // mu / k(eps_f), Kozeny-Carman
    double nbsum = 0.0, fv;
    for (int e = 0; e < g.nd; ++e)
      for (int s = -1; s <= 1; s += 2) {
        const int kd = mom_nb<D>(g, x, e, s, P.u_in, &fv);
        nbsum += kd == 2 ? 2.0 : (kd == 3 ? 0.0 : 1.0);
      }
    double dm, a;
    if (P.simple) {
      dm = (ef * beta + cvis * nbsum) / P.relax_u;
      a = dm / ef;
    } else {
      dm = P.rho / dt + ef * beta + cvis * nbsum;
      a = P.rho / (ef * dt) + beta;
    }
    const double dist = (D == 0 && (x[0] == g.n[0] || x[0] == 0)) ? 0.5 * g.dx : g.dx;
    dmom[f] = dm;
    af[f] = a;
    T[f] = g.S / (a * dist);
  }
}

// Cell gradient of eps (zero-gradient ghosts), |grad eps|, interface normal
// n = -grad/|grad| (0 where |grad| <= 1e-6/dx: below that the direction is set
// by the rounding of eps), and the partial sums of |g|
// and |g| eps (1 - eps) that VoS-psi' fits lambda with.  Central differences,
// or (decentred, a VoS-psi variant of Section 2.4) per direction the one-sided
// difference toward the neighbour of larger eps (ties: the + side), which puts
// the area of a sharp interface in the cell holding the solid.
__global__ void __launch_bounds__(TPB) k_cell_grad(Dev g, int decentred, const double *__restrict__ eps,
                                                   double *__restrict__ gmag, double *__restrict__ n0,
                                                   double *__restrict__ n1, double *__restrict__ n2,
                                                   double *__restrict__ part)
{
  const double tau = 1e-6 / g.dx;
  double s_num = 0.0, s_den = 0.0;
  for (unsigned id = xbeg(g.nc); id < xend(g.nc); id += xstride()) {
    int x[3];
    unflat(g.n, id, x);
    double gv[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < g.nd; ++d) {
      const unsigned st = dstride(g.n, d);
      const double em = x[d] > 0 ? eps[id - st] : eps[id];
      const double ep = x[d] < g.n[d] - 1 ? eps[id + st] : eps[id];
      if (decentred) {
        const double e0 = eps[id];
        gv[d] = em > ep ? (e0 - em) / g.dx : (ep - e0) / g.dx;
      } else {
        gv[d] = (ep - em) / (2.0 * g.dx);
      }
    }
    const double gm = sqrt(gv[0] * gv[0] + gv[1] * gv[1] + gv[2] * gv[2]);
    gmag[id] = gm;
    const double inv = gm > tau ? -1.0 / gm : 0.0;
    n0[id] = gv[0] * inv;
    n1[id] = gv[1] * inv;
    if (g.nd == 3) n2[id] = gv[2] * inv;
    const double e = eps[id];
    s_num += gm;
    s_den += gm * e * (1.0 - e);
  }
  const double v[2] = {s_num, s_den};
  write_partials<2>(v, part);
}

// Reactive face velocity w = kc * (n_lo + n_hi)/2 . e_D * S on interior faces, 0 on the boundary.
template <int D>
__global__ void __launch_bounds__(TPB) k_face_w(Dev g, double kc, const double *__restrict__ nD, double *__restrict__ w)
{
  for (unsigned f = xbeg(g.nf[D]); f < xend(g.nf[D]); f += xstride()) {
    int x[3];
    unflat(g.fd[D], f, x);
    const int q = x[D];
    if (q == 0 || q == g.n[D]) { w[f] = 0.0; continue; }
    const unsigned c = cidx(g, x[0], x[1], x[2]);
    const unsigned st = dstride(g.n, D);
    w[f] = kc * 0.5 * (nD[c - st] + nD[c]) * g.S;
  }
}

// Pressure diagonal: sum of the transmissibilities of the cell's faces.
__global__ void __launch_bounds__(TPB) k_pdiag(Dev g, const double *__restrict__ T0, const double *__restrict__ T1,
                                               const double *__restrict__ T2, double *__restrict__ pd)
{
  for (unsigned id = xbeg(g.nc); id < xend(g.nc); id += xstride()) {
    int x[3];
    unflat(g.n, id, x);
    double s = T0[fidx(g, 0, x[0], x[1], x[2])] + T0[fidx(g, 0, x[0] + 1, x[1], x[2])] +
               T1[fidx(g, 1, x[0], x[1], x[2])] + T1[fidx(g, 1, x[0], x[1] + 1, x[2])];
    if (g.nd == 3) s += T2[fidx(g, 2, x[0], x[1], x[2])] + T2[fidx(g, 2, x[0], x[1], x[2] + 1)];
    pd[id] = s;
  }
}

// lambda for VoS-psi' (4 when the denominator vanishes or for the other models).
__global__ void k_lambda(const double *__restrict__ part, int nb, int model, double *__restrict__ out)
{
  const double num = sum_partials(part, 0, nb);
  const double den = sum_partials(part, 1, nb);
  if (threadIdx.x == 0) {
    double lam = 4.0;
    if (model == 2 && den > 0.0) lam = num / den;
    out[0] = lam;
    out[1] = num;
  }
}

// ---------------------------------------------------------------- S2

// u_D / eps_f on face (D, y) of the D face grid.
template <int D>
__device__ __forceinline__ double conv_phi(const Dev &g, const double *eps, const double *uD, const int y[3])
{
  unsigned lo, hi;
  const double ef = face_eps<D>(g, eps, y, &lo, &hi);
  return uD[fidx(g, D, y[0], y[1], y[2])] / ef;
}

// Momentum convection (Eq. momentumDBS), explicit first-order upwind, on the
// interior face (D, x): rho [div(u u / eps)]_f, the eps_f-scaled row's term.
// Control volume: the cell-sized box centred on the face.  Across its faces
// normal to D (at the centres of the two cells) the transport velocity is the
// mean of that cell's two D-faces; across its faces normal to e != D the mean
// of the two e-faces in that plane belonging to the cells on either side of
// the face.  The transported u_D / eps_f is the box's own value when the flux
// leaves it, else the neighbouring D-face's; beyond the domain 0 enters
// (walls and the inlet carry no tangential momentum) and the outlet plane
// takes the own value (zero gradient).
template <int D>
__device__ double conv_face(const Dev &g, const Phys &P, const double *eps, const double *const uu[3], const int x[3])
{
  double flux = 0.0;
  const double own = conv_phi<D>(g, eps, uu[D], x);
  for (int e = 0; e < g.nd; ++e)
    for (int s = -1; s <= 1; s += 2) {
      int xn[3] = {x[0], x[1], x[2]};
      xn[e] += s;
      double U, nb;
      if (e == D) {
        U = 0.5 * (uu[D][fidx(g, D, x[0], x[1], x[2])] + uu[D][fidx(g, D, xn[0], xn[1], xn[2])]);
        nb = conv_phi<D>(g, eps, uu[D], xn);
      } else {
        const int q = x[e] + (s > 0);
        int cl[3] = {x[0], x[1], x[2]}, cu[3] = {x[0], x[1], x[2]};
        cl[D] -= 1;
        cl[e] = q;
        cu[e] = q;
        U = 0.5 * (uu[e][fidx(g, e, cl[0], cl[1], cl[2])] + uu[e][fidx(g, e, cu[0], cu[1], cu[2])]);
        if (xn[e] >= 0 && xn[e] < g.n[e]) nb = conv_phi<D>(g, eps, uu[D], xn);
        else nb = (e == 0 && s > 0) ? own : 0.0;
      }
      const double out = s * U;
      flux += out * (out >= 0.0 ? own : nb);
    }
  return P.rho * flux / g.dx;
}

// Right-hand side of the eps_f-scaled momentum row of component D and the
// initial guess u^n (fixed rows: b = 0, x = 0).  One pass: inertia rho/dt u^n;
// SIMPLE: the relaxation term dmom (1 - relax_u) u^k.  Pressure gradient of
// p^n across the face (p_out beyond the outlet, p_in before the inlet under
// the pressure drive); explicit convection on interior faces when enabled.
template <int D>
__global__ void __launch_bounds__(TPB) k_mom_rhs(Dev g, Phys P, double dt, const double *__restrict__ eps,
                                                 const double *__restrict__ dmom, const double *__restrict__ u0,
                                                 const double *__restrict__ u1, const double *__restrict__ u2,
                                                 const double *__restrict__ pn, double *__restrict__ b,
                                                 double *__restrict__ x0, int start_un)
{
  const double cvis = P.mu / (g.dx * g.dx);
  const double *const uu[3] = {u0, u1, u2};
  const double *un = uu[D];
  for (unsigned f = xbeg(g.nf[D]); f < xend(g.nf[D]); f += xstride()) {
    int x[3];
    unflat(g.fd[D], f, x);
    if (!mom_unknown<D>(g, x)) { b[f] = 0.0; x0[f] = 0.0; continue; }
    unsigned lo, hi;
    const double ef = face_eps<D>(g, eps, x, &lo, &hi);
    double rhs = P.simple ? dmom[f] * (1.0 - P.relax_u) * un[f] : P.rho / dt * un[f];
    if (D == 0 && x[0] == 1 && !g.drive) rhs += cvis * P.u_in;   // the fixed inlet face is a Laplacian neighbour
    const bool outlet = (D == 0 && x[0] == g.n[0]);
    const bool inlet = (D == 0 && x[0] == 0);   // an unknown only under the pressure drive
    double pl, pu, dist;
    if (inlet) {
      pl = P.p_in;
      pu = pn[cidx(g, 0, x[1], x[2])];
      dist = 0.5 * g.dx;
    } else {
      const unsigned st = dstride(g.n, D);
      const unsigned up = cidx(g, outlet ? g.n[0] - 1 : x[0], x[1], x[2]);
      pl = outlet ? pn[up] : pn[up - st];
      pu = outlet ? P.p_out : pn[up];
      dist = outlet ? 0.5 * g.dx : g.dx;
    }
    rhs -= ef * (pu - pl) / dist;
    if (P.convection && !inlet && !outlet) rhs -= conv_face<D>(g, P, eps, uu, x);
    b[f] = rhs;
    if (start_un) x0[f] = un[f];   // else x0 holds an extrapolated start
  }
}

// q = A p for the momentum system of component D (fixed rows: identity), plus
// the partial sums of p.q.
template <int D>
__global__ void __launch_bounds__(TPB) k_mom_apply(Dev g, double cvis, const double *__restrict__ dmom,
                                                   const double *__restrict__ p, double *__restrict__ q,
                                                   double *__restrict__ part, const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  double acc = 0.0;
  for (unsigned f = xbeg(g.nf[D]); f < xend(g.nf[D]); f += xstride()) {
    int x[3];
    unflat(g.fd[D], f, x);
    const bool unk = mom_unknown<D>(g, x);
    // the neighbour values, loaded together (index of a missing one clamped
    // to the face itself, its term dropped by a select in the same order)
    double pn[6];
    bool use[6];
    double fv;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const bool de = e < g.nd;
      const unsigned st = de ? dstride(g.fd[D], e) : 0u;
      use[2 * e] = de && unk && mom_nb<D>(g, x, e, -1, 0.0, &fv) == 0;
      use[2 * e + 1] = de && unk && mom_nb<D>(g, x, e, +1, 0.0, &fv) == 0;
      pn[2 * e] = p[use[2 * e] ? f - st : f];
      pn[2 * e + 1] = p[use[2 * e + 1] ? f + st : f];
    }
    const double pf = p[f];
    double v = dmom[f] * pf;
    if (unk) {
      double nb = 0.0;
#pragma unroll
      for (int k = 0; k < 6; ++k) nb = use[k] ? nb + pn[k] : nb;
      v -= cvis * nb;
    }
    q[f] = v;
    acc += pf * v;
  }
  const double vv[1] = {acc};
  write_partials<1>(vv, part);
}

// Restore the fixed faces of a momentum predictor (inlet u_in, walls 0).
template <int D>
__global__ void __launch_bounds__(TPB) k_mom_fix(Dev g, double u_in, double *__restrict__ u)
{
  for (unsigned f = xbeg(g.nf[D]); f < xend(g.nf[D]); f += xstride()) {
    int x[3];
    unflat(g.fd[D], f, x);
    if (!mom_unknown<D>(g, x)) u[f] = (D == 0 && x[0] == 0) ? u_in : 0.0;
  }
}

// ---------------------------------------------------------------- S3

// Pressure operator q = A p: sum over faces T (p_P - p_N), the outlet face
// contributing T p_P (Dirichlet increment), plus partials of p.q.
__device__ __forceinline__ double papply_cell(const Dev &g, const double *T0, const double *T1, const double *T2,
                                              const double *p, unsigned id, const int x[3])
{
  const double pc = p[id];
  const unsigned f0 = fidx(g, 0, x[0], x[1], x[2]);
  const double tw = T0[f0], te = T0[f0 + 1];
  double v = (tw + te) * pc;
  if (x[0] > 0) v -= tw * p[id - 1];
  if (x[0] < g.n[0] - 1) v -= te * p[id + 1];
  const unsigned f1 = fidx(g, 1, x[0], x[1], x[2]);
  const unsigned sy = (unsigned)g.fd[1][0];
  const double ts = T1[f1], tn = T1[f1 + sy];
  v += (ts + tn) * pc;
  if (x[1] > 0) v -= ts * p[id - g.n[0]];
  if (x[1] < g.n[1] - 1) v -= tn * p[id + g.n[0]];
  if (g.nd == 3) {
    const unsigned f2 = fidx(g, 2, x[0], x[1], x[2]);
    const unsigned sz = (unsigned)g.n[0] * g.n[1];
    const double tb = T2[f2], tt = T2[f2 + sz];
    v += (tb + tt) * pc;
    if (x[2] > 0) v -= tb * p[id - sz];
    if (x[2] < g.n[2] - 1) v -= tt * p[id + sz];
  }
  return v;
}

__global__ void __launch_bounds__(TPB) k_p_apply(Dev g, const double *__restrict__ T0, const double *__restrict__ T1,
                                                 const double *__restrict__ T2, const double *__restrict__ p,
                                                 double *__restrict__ q, double *__restrict__ part,
                                                 const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  double acc = 0.0;
  for (unsigned id = xbeg(g.nc); id < xend(g.nc); id += xstride()) {
    int x[3];
    unflat(g.n, id, x);
    const double v = papply_cell(g, T0, T1, T2, p, id, x);
    q[id] = v;
    acc += p[id] * v;
  }
  const double vv[1] = {acc};
  write_partials<1>(vv, part);
}

// b = A p^n - div(u*) (+ the continuity source of Eq. contDBS, src_c Rbar V,
// with the lagged rates rsrc when given; partial sums of it in part).
__global__ void __launch_bounds__(TPB) k_p_rhs(Dev g, const double *__restrict__ T0, const double *__restrict__ T1,
                                               const double *__restrict__ T2, const double *__restrict__ pn,
                                               const double *__restrict__ u0, const double *__restrict__ u1,
                                               const double *__restrict__ u2, double *__restrict__ b,
                                               const double *__restrict__ rsrc, double src_c,
                                               double *__restrict__ part)
{
  double ssum = 0.0;
  for (unsigned id = xbeg(g.nc); id < xend(g.nc); id += xstride()) {
    int x[3];
    unflat(g.n, id, x);
    const double ap = papply_cell(g, T0, T1, T2, pn, id, x);
    const unsigned f0 = fidx(g, 0, x[0], x[1], x[2]);
    const unsigned f1 = fidx(g, 1, x[0], x[1], x[2]);
    double div = (u0[f0 + 1] - u0[f0]) + (u1[f1 + g.fd[1][0]] - u1[f1]);
    if (g.nd == 3) {
      const unsigned f2 = fidx(g, 2, x[0], x[1], x[2]);
      div += u2[f2 + (unsigned)g.n[0] * g.n[1]] - u2[f2];
    }
    double v = ap - div * g.S;
    if (rsrc) {
      const double sv = src_c * rsrc[id] * g.V;
      v += sv;
      ssum += sv;
    }
    b[id] = v;
  }
  if (rsrc) {
    const double vv[1] = {ssum};
    write_partials<1>(vv, part);
  }
}

// ---------------------------------------------------------------- S4

// u = u* - [(p - p^n)_hi - (p - p^n)_lo] / (af d_f) on the momentum unknowns
// (the increment vanishes at the Dirichlet outlet, and at the inlet under the
// pressure drive).
template <int D>
__global__ void __launch_bounds__(TPB) k_correct(Dev g, const double *__restrict__ ustar, const double *__restrict__ af,
                                                 const double *__restrict__ p, const double *__restrict__ pn,
                                                 double *__restrict__ u)
{
  for (unsigned f = xbeg(g.nf[D]); f < xend(g.nf[D]); f += xstride()) {
    int x[3];
    unflat(g.fd[D], f, x);
    if (!mom_unknown<D>(g, x)) { u[f] = ustar[f]; continue; }
    const bool outlet = (D == 0 && x[0] == g.n[0]);
    if (D == 0 && x[0] == 0) {
      const unsigned c0 = cidx(g, 0, x[1], x[2]);
      u[f] = ustar[f] - ((p[c0] - pn[c0]) - 0.0) / (af[f] * (0.5 * g.dx));
      continue;
    }
    const unsigned st = dstride(g.n, D);
    const unsigned up = cidx(g, outlet ? g.n[0] - 1 : x[0], x[1], x[2]);
    const unsigned lo = outlet ? up : up - st;
    const double dpl = p[lo] - pn[lo];
    const double dpu = outlet ? 0.0 : p[up] - pn[up];
    const double dist = outlet ? 0.5 * g.dx : g.dx;
    u[f] = ustar[f] - (dpu - dpl) / (af[f] * dist);
  }
}

// ---------------------------------------------------------------- S5

// van Leer correction of phi on the interior face between cells lo and hi =
// lo + st along direction d (cell coordinate of hi: xh), for face velocity vel.
__device__ __forceinline__ double face_corr(const double *phi, unsigned lo, unsigned st, int xh, int nd_, double vel)
{
  const unsigned hi = lo + st;
  if (vel >= 0.0) {
    const double pc = phi[lo], pd = phi[hi];
    const double pu = (xh - 2 >= 0) ? phi[lo - st] : pc;
    return vanleer_corr(pu, pc, pd);
  }
  const double pc = phi[hi], pd = phi[lo];
  const double pu = (xh + 1 < nd_) ? phi[hi + st] : pc;
  return vanleer_corr(pu, pc, pd);
}

// Transport rows of every cell, scaled by their diagonal: off-diagonals
// (-x,+x,-y,+y,-z,+z) and right-hand side.  Convection is upwind with the van
// Leer correction lagged on c^n (deferred correction), diffusion eps_f D S/dx,
// the iVoS acid sink eps_P sum_f w_f c^R_f (same treatment along w), the psi
// sink kc psi |grad eps| V c_P (implicit).  Inlet: Dirichlet c_in; outlet:
// zero gradient; walls: no flux.
// face_corr on the face between the cell (coordinate x along the direction, n
// cells) and its neighbour on side s, from the five values of phi at offsets
// -2..+2 along the direction (loaded beforehand; an offset outside the grid
// holds any value, never used): the same upwind, central and downwind values
// as face_corr, so the same correction.
__device__ __forceinline__ double face_corr5(const double (&ph)[5], int s, int x, int n, double vel)
{
  if (s > 0) {   // lo = the cell, hi = x + 1
    if (vel >= 0.0) return vanleer_corr(x - 1 >= 0 ? ph[1] : ph[2], ph[2], ph[3]);
    return vanleer_corr(x + 2 < n ? ph[4] : ph[3], ph[3], ph[2]);
  }
  // lo = x - 1, hi = the cell
  if (vel >= 0.0) return vanleer_corr(x - 2 >= 0 ? ph[0] : ph[1], ph[1], ph[2]);
  return vanleer_corr(x + 1 < n ? ph[3] : ph[2], ph[2], ph[1]);
}

__global__ void __launch_bounds__(TPB) k_adr_assemble(Dev g, Phys P, const double *__restrict__ eps,
                                                      const double *__restrict__ u0, const double *__restrict__ u1,
                                                      const double *__restrict__ u2, const double *__restrict__ w0,
                                                      const double *__restrict__ w1, const double *__restrict__ w2,
                                                      const double *__restrict__ cold, const double *__restrict__ gmag,
                                                      const double *__restrict__ lam, double *__restrict__ off,
                                                      double *__restrict__ b, double *__restrict__ dg,
                                                      double *__restrict__ dif, int vl, double dt,
                                                      const double *__restrict__ eps_prev,
                                                      const double *__restrict__ c0)
{
  const double *uu[3] = {u0, u1, u2};
  const double *ww[3] = {w0, w1, w2};
  const double lambda = lam[0];
  for (unsigned id = xbeg(g.nc); id < xend(g.nc); id += xstride()) {
    int x[3];
    unflat(g.n, id, x);
    // every value the row needs, loaded before any arithmetic (indices clamped
    // into the arrays; the ones a boundary does not use are dropped below)
    const double ep = eps[id];
    double uf[3][2], wf[3][2], enb[3][2], ph[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (d >= g.nd) {   // 2-D: no z faces (block-uniform)
        uf[d][0] = uf[d][1] = wf[d][0] = wf[d][1] = enb[d][0] = enb[d][1] = 0.0;
        for (int k = 0; k < 5; ++k) ph[d][k] = 0.0;
        continue;
      }
      const int xd = x[d], nd_ = g.n[d];
      const unsigned st = dstride(g.n, d);
      const unsigned flo = fidx(g, d, x[0], x[1], x[2]);
      const unsigned fhi = flo + dstride(g.fd[d], d);
      uf[d][0] = uu[d][flo];
      uf[d][1] = uu[d][fhi];
      wf[d][0] = ww[d][flo];
      wf[d][1] = ww[d][fhi];
      enb[d][0] = eps[xd > 0 ? id - st : id];
      enb[d][1] = eps[xd + 1 < nd_ ? id + st : id];
#pragma unroll
      for (int k = -2; k <= 2; ++k) {
        const bool in = xd + k >= 0 && xd + k < nd_;
        ph[d][k + 2] = cold[in ? (k < 0 ? id - (unsigned)(-k) * st : id + (unsigned)k * st) : id];
      }
    }
    const double gm = gmag[id];
    const double epv = P.transient ? eps_prev[id] : 0.0, c0v = P.transient ? c0[id] : 0.0;
    const double cv = cold[id];
    double diag = 0.0, rhs = 0.0, o[6] = {0, 0, 0, 0, 0, 0}, od[6] = {0, 0, 0, 0, 0, 0};
    for (int d = 0; d < g.nd; ++d) {
      for (int s = -1; s <= 1; s += 2) {
        const int xf_d = x[d] + (s > 0);
        const double ufc = uf[d][s > 0];
        const double Fo = s * g.S * ufc;
        const int slot = 2 * d + (s > 0);
        if (xf_d > 0 && xf_d < g.n[d]) {
          if (Fo >= 0.0) diag += Fo; else o[slot] += Fo;
          if (vl) rhs -= Fo * face_corr5(ph[d], s, x[d], g.n[d], ufc);
          const double G = P.D * 0.5 * (ep + enb[d][s > 0]) * g.S / g.dx;
          diag += G;
          o[slot] -= G;
          od[slot] = -G;
          if (P.model == 0) {
            const double wfc = wf[d][s > 0];
            const double k = P.zeta * ep * (s * wfc);
            if (k >= 0.0) diag += k; else o[slot] += k;
            if (vl) rhs -= k * face_corr5(ph[d], s, x[d], g.n[d], wfc);
          }
        } else if (d == 0 && xf_d == 0) {
          if (Fo < 0.0) rhs -= Fo * P.c_in; else diag += Fo;
          const double G = P.D * ep * g.S / (0.5 * g.dx);
          diag += G;
          rhs += G * P.c_in;
        } else if (d == 0) {
          diag += Fo;
        }
      }
    }
    if (P.model != 0) {
      const double psi = P.psi_kind == 1 ? 1.0 : lambda * ep * (1.0 - ep);
      diag += P.zeta * P.kc * psi * gm * g.V;
    }
    if (P.transient) {
      diag += ep * g.V / dt;
      rhs += epv * c0v * g.V / dt;
    }
    if (P.simple && P.relax_c < 1.0) {
      const double dr = diag / P.relax_c;
      rhs += (dr - diag) * cv;
      diag = dr;
    }
    const double inv = 1.0 / diag;
    for (int k = 0; k < 2 * g.nd; ++k) off[(size_t)k * g.nc + id] = o[k] * inv;
    for (int k = 0; k < 2 * g.nd; ++k) dif[(size_t)k * g.nc + id] = od[k];
    b[id] = rhs * inv;
    dg[id] = diag;
  }
}

// splitmix64 (Steele, Lea & Flood 2014) of counter i, as a double in [-1, 1).
__device__ __forceinline__ double splitmix_unit(unsigned long long i)
{
  unsigned long long z = (i + 1ULL) * 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  return (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// y = A x for the scaled transport rows (unit diagonal), with up to two dot
// partials: slot 0 <y, w>, slot 1 <y, y> (NDOT = 1 or 2, w may be y's partner).
// HW: w is BiCGStab's shadow residual splitmix_unit(cell), formed in place
// (the w argument is not read).
template <int NDOT, bool HW = false>
__global__ void __launch_bounds__(TPB) k_adr_apply(Dev g, const double *__restrict__ off, const double *__restrict__ xv,
                                                   double *__restrict__ y, const double *__restrict__ w,
                                                   double *__restrict__ part, const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  double d0 = 0.0, d1 = 0.0;
  const unsigned sy = (unsigned)g.n[0], sz = (unsigned)g.n[0] * g.n[1];
  for (unsigned id = xbeg(g.nc); id < xend(g.nc); id += xstride()) {
    int x[3];
    unflat(g.n, id, x);
    // every load issued together (a missing neighbour's index clamped to the
    // cell itself, its term dropped by a select in the same order: -x, +x,
    // -y, +y, -z, +z; a 2-D grid has no z neighbours)
    const bool h[6] = {x[0] > 0, x[0] < g.n[0] - 1, x[1] > 0, x[1] < g.n[1] - 1, x[2] > 0, x[2] < g.n[2] - 1};
    const unsigned nb[6] = {h[0] ? id - 1 : id, h[1] ? id + 1 : id, h[2] ? id - sy : id,
                            h[3] ? id + sy : id, h[4] ? id - sz : id, h[5] ? id + sz : id};
    double xn[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, o[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      if (k >= 4 && g.nd != 3) continue;   // uniform: a 2-D grid reads no z slots
      xn[k] = xv[nb[k]];
      o[k] = off[(size_t)k * g.nc + id];
    }
    double v = xv[id];
#pragma unroll
    for (int k = 0; k < 6; ++k) v = h[k] ? v + o[k] * xn[k] : v;
    y[id] = v;
    d0 += v * (HW ? splitmix_unit(id) : w[id]);
    if (NDOT == 2) d1 += v * v;
  }
  if (NDOT == 1) { const double vv[1] = {d0}; write_partials<1>(vv, part); }
  else { const double vv[2] = {d0, d1}; write_partials<2>(vv, part); }
}

// ---------------------------------------------------------------- S6 / S7

// Reaction rate per cell.  iVoS (Eq. RfiVoS): Rbar V = eps_P sum_f w_f c^R_f -
// sum_f w_f (eps c)^R_f with c^R_f the transport solve's face values (upwind
// of c^{n+1} + van Leer correction lagged on c^n) and (eps c)^R_f the van
// Leer face value of eps^n c^{n+1}; the acid sink is the first term.
// psi models (Eq. RfVoSpsi): Rbar = kc psi |grad eps| c, psi = lambda eps(1-eps)
// or 1.  Per block, the largest |Vm Rbar| over the cells free to move by more
// than deps_max (pmax).
__global__ void __launch_bounds__(TPB) k_react(Dev g, Phys P, const double *__restrict__ eps,
                                               const double *__restrict__ c, const double *__restrict__ cold,
                                               const double *__restrict__ w0, const double *__restrict__ w1,
                                               const double *__restrict__ w2, const double *__restrict__ gmag,
                                               const double *__restrict__ lam, double *__restrict__ rbar,
                                               double *__restrict__ part, double *__restrict__ pmax, double deps_max)
{
  const double *ww[3] = {w0, w1, w2};
  const double lambda = lam[0];
  double s_sink = 0.0, s_rate = 0.0, mrate = 0.0;
  for (unsigned id = xbeg(g.nc); id < xend(g.nc); id += xstride()) {
    int x[3];
    unflat(g.n, id, x);
    const double ep = eps[id];
    double R, sk;
    if (P.model == 0) {
      double t1 = 0.0, t2 = 0.0;
      for (int d = 0; d < g.nd; ++d) {
        const unsigned st = dstride(g.n, d);
        const int xd = x[d], nd_ = g.n[d];
        // w on the cell's two faces, eps, c and c^n at offsets -2..+2 along d,
        // all loaded before the arithmetic (indices clamped into the grid; a
        // value outside it is never used)
        const unsigned flo = fidx(g, d, x[0], x[1], x[2]);
        const double wlo = ww[d][flo], whi = ww[d][flo + dstride(g.fd[d], d)];
        double e5[5], c5[5], o5[5];
#pragma unroll
        for (int k = -2; k <= 2; ++k) {
          const bool in = xd + k >= 0 && xd + k < nd_;
          const unsigned j = in ? (k < 0 ? id - (unsigned)(-k) * st : id + (unsigned)k * st) : id;
          e5[k + 2] = eps[j];
          c5[k + 2] = c[j];
          o5[k + 2] = cold[j];
        }
        for (int s = -1; s <= 1; s += 2) {
          const int xf_d = xd + (s > 0);
          if (xf_d == 0 || xf_d == nd_) continue;
          const double wf = s > 0 ? whi : wlo;
          const double wo = s * wf;
          // the face's lower and upper cells in the five-value window
          const int L = s > 0 ? 2 : 1, H = L + 1;
          // upwind cell along w for c; van Leer of c^n lagged, and of q = eps c
          const double cR = c5[wf >= 0.0 ? L : H] + face_corr5(o5, s, xd, nd_, wf);
          double qU, qC, qD;
          if (wf >= 0.0) {
            qC = e5[L] * c5[L];
            qD = e5[H] * c5[H];
            qU = (xf_d - 2 >= 0) ? e5[L - 1] * c5[L - 1] : qC;
          } else {
            qC = e5[H] * c5[H];
            qD = e5[L] * c5[L];
            qU = (xf_d + 1 < nd_) ? e5[H + 1] * c5[H + 1] : qC;
          }
          const double qR = qC + vanleer_corr(qU, qC, qD);
          t1 += wo * cR;
          t2 += wo * qR;
        }
      }
      sk = ep * t1;
      R = sk - t2;
    } else {
      const double psi = P.psi_kind == 1 ? 1.0 : lambda * ep * (1.0 - ep);
      sk = P.kc * psi * gmag[id] * c[id] * g.V;
      R = sk;
    }
    const double rb = R / g.V;
    rbar[id] = rb;
    // Appendix D's bound looks at the cells the clip does not hold within
    // deps_max of their bound (a cell closer to it changes by at most that)
    const double r = P.Vm * rb;
    const double room = r > 0.0 ? 1.0 - ep : ep - P.eps_min;
    if (room > deps_max) mrate = fmax(mrate, fabs(r));
    s_sink += sk;
    s_rate += R;
  }
  const double v[2] = {s_sink, s_rate};
  write_partials<2>(v, part);
  __shared__ double lds[TPB / 64];
  const double m = block_max(mrate, lds);
  if (threadIdx.x == 0) pmax[blockIdx.x] = m;
}

// Time step of the solid update (Appendix D): min(dt, deps_max / max |Vm Rbar|)
// from k_react's per-block maxima; dt when no cell reacts.
__global__ void k_solid_dt(const double *__restrict__ pmax, int nb, double dt, double deps_max,
                           double *__restrict__ out)
{
  const double m = max_partials(pmax, 0, nb);
  if (threadIdx.x != 0) return;
  double dts = dt;
  if (m > 0.0) {
    const double lim = deps_max / m;
    dts = lim < dt ? lim : dt;
  }
  out[0] = dts;
}

// Solid update eps <- clip(eps + dt Vm Rbar, eps_min, 1) (Eq. mbs) and the
// diagnostic sums: 0 clipped, 1 d(eps)V, 2 solid volume, 3 sum eps, 4 inlet
// acid flux, 5 outlet acid flux, 6 inlet p, 7 sum c|g|V, 8 sum eps c V,
// 9 sum |g| V, 10 inlet volume flux, 11 transient storage sum
// (eps c - eps_prev c0) V / dt; max |d eps| goes to the separate max slot
// array.  Transient: eps_prev takes eps^n for the next step's storage term.
__global__ void __launch_bounds__(TPB) k_eps_update(Dev g, Phys P, double dt_arg, const double *__restrict__ dtp,
                                                    int freeze, double *__restrict__ eps,
                                                    const double *__restrict__ rbar, const double *__restrict__ c,
                                                    const double *__restrict__ p, const double *__restrict__ u0,
                                                    const double *__restrict__ gmag, double *__restrict__ part,
                                                    double *__restrict__ part_max, double *__restrict__ eps_prev,
                                                    const double *__restrict__ c0)
{
  double v[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  double mx = 0.0;
  const double dt = dtp ? dtp[0] : dt_arg;   // the shortened solid step when there is one
  for (unsigned id = xbeg(g.nc); id < xend(g.nc); id += xstride()) {
    int x[3];
    unflat(g.n, id, x);
    const double e0 = eps[id], cc = c[id];
    if (x[0] == 0) {
      const double ui = u0[fidx(g, 0, 0, x[1], x[2])];
      v[4] += g.S * ui * (ui > 0.0 ? P.c_in : cc) + P.D * e0 * g.S / (0.5 * g.dx) * (P.c_in - cc);
      v[6] += p[id];
      v[10] += g.S * ui;
    }
    if (x[0] == g.n[0] - 1) v[5] += g.S * u0[fidx(g, 0, g.n[0], x[1], x[2])] * cc;
    v[7] += cc * gmag[id] * g.V;
    v[8] += e0 * cc * g.V;
    v[9] += gmag[id] * g.V;
    if (P.transient) {
      v[11] += (e0 * cc - eps_prev[id] * c0[id]) * g.V / dt_arg;
      eps_prev[id] = e0;
    }
    double e1c = e0;
    if (!freeze) {
      const double e1 = e0 + dt * P.Vm * rbar[id];
      e1c = e1 < P.eps_min ? P.eps_min : (e1 > 1.0 ? 1.0 : e1);
      v[0] += (e1 - e1c) * g.V;
      v[1] += (e1c - e0) * g.V;
      mx = fmax(mx, fabs(e1c - e0));
      eps[id] = e1c;
    }
    v[2] += (1.0 - e1c) * g.V;
    v[3] += e1c;
  }
  write_partials<12>(v, part);
  __shared__ double lds[TPB / 64];
  const double m = block_max(mx, lds);
  if (threadIdx.x == 0) part_max[blockIdx.x] = m;
}

// ---------------------------------------------------------------- Krylov vector kernels

// r = b - q; z = r / dg; p = z; partials r.z, b.b/dg.
__global__ void __launch_bounds__(TPB) k_cg_init(unsigned n, const double *__restrict__ b, const double *__restrict__ q,
                                                 const double *__restrict__ dg, double *__restrict__ r,
                                                 double *__restrict__ z, double *__restrict__ p, int jacobi,
                                                 double *__restrict__ part)
{
  double rz = 0.0, bn = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double d = dg[i];
    const double rr = b[i] - q[i];
    r[i] = rr;
    if (jacobi) { const double zz = rr / d; z[i] = zz; p[i] = zz; }
    rz += rr * rr / d;
    bn += b[i] * b[i] / d;
  }
  const double v[2] = {rz, bn};
  write_partials<2>(v, part);
}

// x += alpha p; r -= alpha q; (jacobi) z = r/dg; partial sum r^2/dg.
__global__ void __launch_bounds__(TPB) k_cg_xr(unsigned n, const double *__restrict__ p, const double *__restrict__ q,
                                               const double *__restrict__ dg, double *__restrict__ x,
                                               double *__restrict__ r, double *__restrict__ z, int jacobi,
                                               double *__restrict__ part, const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  const double alpha = sc[S_ALPHA];
  double res = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    x[i] += alpha * p[i];
    const double rr = r[i] - alpha * q[i];
    r[i] = rr;
    const double d = dg[i];
    if (jacobi) z[i] = rr / d;
    res += rr * rr / d;
  }
  const double v[1] = {res};
  write_partials<1>(v, part);
}

// Partials z.r and z.q (flexible CG after a non-Jacobi preconditioner); with
// p (the start of a solve) also the first direction p = z.
__global__ void __launch_bounds__(TPB) k_cg_zdots(unsigned n, const double *__restrict__ z, const double *__restrict__ r,
                                                  const double *__restrict__ q, double *__restrict__ part,
                                                  const double *__restrict__ sc, double *__restrict__ p = nullptr)
{
  if (sc[S_CONV] != 0.0) return;
  double zr = 0.0, zq = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double zi = z[i];
    if (p) p[i] = zi;
    zr += zi * r[i];
    zq += zi * q[i];
  }
  const double v[2] = {zr, zq};
  write_partials<2>(v, part);
}

// p = z + beta p.
__global__ void __launch_bounds__(TPB) k_cg_p(unsigned n, const double *__restrict__ z, double *__restrict__ p,
                                              const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  const double beta = sc[S_BETA];
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) p[i] = z[i] + beta * p[i];
}

// One-block scalar updates of the CG recurrences.
//  op 0 (init):  rz, bn2 from partials (slot 0 r.z or r^2/dg, slot 1 b^2/dg); conv test.
//  op 1 (alpha): alpha = rz / p.q.
//  op 2 (beta, Jacobi): res2 = r^2/dg (= r.z); beta = res2 / rz; rz = res2; conv test.
//  op 3 (residual, flexible): res2 from partials; conv test.
//  op 4 (beta, flexible): rz_new = z.r; beta = -alpha z.q / rz; rz = rz_new.
//  op 5 (init rz, flexible): rz = z.r.
__global__ void k_cg_scal(int op, const double *__restrict__ part, int nb, double rtol2, double *__restrict__ sc)
{
  if (op != 0 && sc[S_CONV] != 0.0) return;
  const double a = sum_partials(part, 0, nb);
  const double b = (op == 0 || op == 4) ? sum_partials(part, 1, nb) : 0.0;
  if (threadIdx.x != 0) return;
  switch (op) {
    case 0:
      sc[S_RZ] = a; sc[S_RES2] = a; sc[S_RES0] = a; sc[S_BN2] = b; sc[S_TOL2] = rtol2 * b; sc[S_ITS] = 0.0;
      sc[S_CONV] = (a <= rtol2 * b || a == 0.0) ? 1.0 : 0.0;
      sc[S_BAD] = 0.0;
      break;
    case 1:
      if (a > 0.0) sc[S_ALPHA] = sc[S_RZ] / a;
      else { sc[S_ALPHA] = 0.0; sc[S_BAD] = 1.0; sc[S_CONV] = 1.0; }
      break;
    case 2:
      sc[S_RES2] = a;
      sc[S_ITS] += 1.0;
      sc[S_BETA] = a / sc[S_RZ];
      sc[S_RZ] = a;
      if (a <= sc[S_TOL2] || !(a == a)) sc[S_CONV] = 1.0;
      break;
    case 3:
      sc[S_RES2] = a;
      sc[S_ITS] += 1.0;
      if (a <= sc[S_TOL2] || !(a == a)) sc[S_CONV] = 1.0;
      break;
    case 4:
      sc[S_BETA] = -sc[S_ALPHA] * b / sc[S_RZ];
      sc[S_RZ] = a;
      break;
    case 5:
      sc[S_RZ] = a;
      break;
  }
}

// ---------------------------------------------------------------- BiCGStab vector kernels

// r = b - y; rh = fixed pseudo-random shadow residual (global support, so
// rh.r cannot vanish as a cold-start residual travels downstream); p = v = 0;
// partials b.b, r.r, rh.r
__global__ void __launch_bounds__(TPB) k_bi_init(unsigned n, const double *__restrict__ b, const double *__restrict__ y,
                                                 double *__restrict__ r, double *__restrict__ rh, double *__restrict__ p,
                                                 double *__restrict__ v, double *__restrict__ part)
{
  double bb = 0.0, rr = 0.0, hr = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double ri = b[i] - y[i];
    const double h = splitmix_unit(i);
    r[i] = ri; p[i] = 0.0; v[i] = 0.0;
    if (rh) rh[i] = h;
    bb += b[i] * b[i];
    rr += ri * ri;
    hr += h * ri;
  }
  const double vv[3] = {bb, rr, hr};
  write_partials<3>(vv, part);
}

// p = r + beta (p - omega v); pd = p dg (the preconditioner's input; not
// stored when pd is null)
__global__ void __launch_bounds__(TPB) k_bi_p(unsigned n, const double *__restrict__ r, const double *__restrict__ v,
                                              double *__restrict__ p, double *__restrict__ pd,
                                              const double *__restrict__ dg, const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  const double beta = sc[S_BETA], om = sc[S_OMEGA];
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double pi = r[i] + beta * (p[i] - om * v[i]);
    p[i] = pi;
    if (pd) pd[i] = pi * dg[i];
  }
}

// s = r - alpha v, sd = s dg (the preconditioner's input; not stored when sd
// is null), partial s.s
__global__ void __launch_bounds__(TPB) k_bi_s(unsigned n, const double *__restrict__ r, const double *__restrict__ v,
                                              double *__restrict__ s, double *__restrict__ sd,
                                              const double *__restrict__ dg, double *__restrict__ part,
                                              const double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  const double al = sc[S_ALPHA];
  double ss = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double si = r[i] - al * v[i];
    s[i] = si;
    if (sd) sd[i] = si * dg[i];
    ss += si * si;
  }
  const double vv[1] = {ss};
  write_partials<1>(vv, part);
}

// x += alpha ph + omega sh; r = s - omega t (or only x += alpha ph after an
// early exit on s); partials r.r, rh.r with rh the shadow residual
// splitmix_unit(i), formed in place.  ph, sh: preconditioned directions.
__global__ void __launch_bounds__(TPB) k_bi_xr(unsigned n, const double *__restrict__ ph, const double *__restrict__ sh,
                                               const double *__restrict__ s, const double *__restrict__ t,
                                               double *__restrict__ x, double *__restrict__ r,
                                               double *__restrict__ part, double *__restrict__ sc)
{
  if (sc[S_CONV] != 0.0) return;
  const double al = sc[S_ALPHA], om = sc[S_OMEGA];
  const bool half = sc[S_SHALF] != 0.0;
  double rr = 0.0, rhr = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    if (half) { x[i] += al * ph[i]; continue; }
    x[i] += al * ph[i] + om * sh[i];
    const double ri = s[i] - om * t[i];
    r[i] = ri;
    rr += ri * ri;
    rhr += splitmix_unit(i) * ri;
  }
  const double vv[2] = {rr, rhr};
  write_partials<2>(vv, part);
}

// Partial sums of |b - y|^2 (y = A x): the true residual of a BiCGStab iterate.
__global__ void __launch_bounds__(TPB) k_bi_true_res(unsigned n, const double *__restrict__ b,
                                                     const double *__restrict__ y, double *__restrict__ part)
{
  double a = 0.0;
  for (unsigned i = xbeg(n); i < xend(n); i += xstride()) {
    const double r = b[i] - y[i];
    a += r * r;
  }
  const double vv[1] = {a};
  write_partials<1>(vv, part);
}

__global__ void k_bi_true_scal(const double *__restrict__ part, int nb, double *__restrict__ sc)
{
  const double a = sum_partials(part, 0, nb);
  if (threadIdx.x == 0) sc[S_TRUE] = a;
}

// BiCGStab scalars.
//  op 0 (init): bn2 = b.b, res2 = r.r, rho = rh.r, alpha = omega = 1, beta = 0; conv test.
//  op 1 (alpha): alpha = rho / rh.v (partial slot 0).
//  op 2 (s test): s.s <= tol2 -> half step then converge.
//  op 3 (omega): omega = t.s / t.t (slots 0, 1).
//  op 4 (after xr): res2 = r.r, rho_new = rh.r; conv test; beta = (rho_new/rho)(alpha/omega).
__global__ void k_bi_scal(int op, const double *__restrict__ part, int nb, double rtol2, double *__restrict__ sc)
{
  if (op != 0 && sc[S_CONV] != 0.0) return;
  const double a = sum_partials(part, 0, nb);
  const double b = (op == 0 || op == 3 || op == 4) ? sum_partials(part, 1, nb) : 0.0;
  const double c3 = (op == 0) ? sum_partials(part, 2, nb) : 0.0;
  if (threadIdx.x != 0) return;
  switch (op) {
    case 0: {
      sc[S_BN2] = a; sc[S_RES2] = b; sc[S_RES0] = b; sc[S_TOL2] = rtol2 * a; sc[S_ITS] = 0.0; sc[S_BAD] = 0.0;
      sc[S_ALPHA] = 1.0; sc[S_OMEGA] = 1.0; sc[S_SHALF] = 0.0;
      sc[S_CONV] = (b <= rtol2 * a || b == 0.0) ? 1.0 : 0.0;
      // first direction p = r: beta = 0, rho = rh.r
      sc[S_BETA] = 0.0;
      sc[S_RHO] = c3;
      if (c3 == 0.0 && sc[S_CONV] == 0.0) { sc[S_BAD] = 1.0; sc[S_CONV] = 1.0; }
      break;
    }
    case 1:
      if (a != 0.0) sc[S_ALPHA] = sc[S_RHO] / a;
      else { sc[S_BAD] = 1.0; sc[S_CONV] = 1.0; }
      break;
    case 2:
      if (a <= sc[S_TOL2]) { sc[S_SHALF] = 1.0; sc[S_RES2] = a; }
      break;
    case 3:
      if (sc[S_SHALF] == 0.0) {
        if (b != 0.0) sc[S_OMEGA] = a / b;
        else { sc[S_BAD] = 1.0; sc[S_CONV] = 1.0; }
      }
      break;
    case 4: {
      sc[S_ITS] += 1.0;
      if (sc[S_SHALF] != 0.0) { sc[S_CONV] = 1.0; break; }
      sc[S_RES2] = a;
      if (a <= sc[S_TOL2] || !(a == a)) { sc[S_CONV] = 1.0; break; }
      if (b == 0.0 || sc[S_OMEGA] == 0.0) { sc[S_BAD] = 1.0; sc[S_CONV] = 1.0; break; }
      sc[S_BETA] = (b / sc[S_RHO]) * (sc[S_ALPHA] / sc[S_OMEGA]);
      sc[S_RHO] = b;
      break;
    }
  }
}

}  // namespace vos
