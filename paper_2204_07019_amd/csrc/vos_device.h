// vos_device.h -- device-side helpers shared by the gfx950 kernels of the VoS step.
//
// Layout: cells x fastest, id = i + nx*(j + ny*k).  Face grid of direction d
// has dims n + e_d; face (d, x) lies between cells x - e_d and x.
#pragma once
#include <hip/hip_runtime.h>

namespace vos {

constexpr int TPB = 256;         // threads per block of every sweep (4 wave64s)
constexpr int MAXB = 4096;       // blocks of a grid-stride sweep == partial-sum slots per quantity
constexpr int NSLOT = 16;        // partial-sum quantities one sweep may produce

struct Dev {
  int n[3];
  int nd;                        // 2 (nz == 1) or 3
  int drive;                     // 1: inlet pressure drive (the inlet x-faces are momentum unknowns)
  int fd[3][3];                  // face-grid dims
  unsigned nc;
  unsigned nf[3];
  double dx, S, V;
};

struct Phys {
  double mu, rho, D, k0, kc, Vm, zeta, c_in, eps_min, u_in, p_out;
  int model;
  double p_in;                   // inlet pressure (pressure drive)
  int convection;                // explicit upwind momentum convection
  int grad_scheme;               // 0 central, 1 decentred gradient of eps (VoS-psi variants)
  int psi_kind;                  // 0: psi = lambda eps (1 - eps); 1: psi = 1
  int transient;                 // storage d(eps c)/dt and the continuity source
  double Vm_f;                   // M_ws / rho of the fluid
  int simple;                    // quasi-static SIMPLE loop: steady momentum with relaxation
  double relax_u, relax_c;       // its implicit under-relaxation factors
};

__device__ __forceinline__ unsigned gtid() { return blockIdx.x * blockDim.x + threadIdx.x; }

// a b rounded to FP64 on its own: the product never enters a fused
// multiply-add with the arithmetic that consumes it (so it equals the same
// product stored to memory and read back).
__device__ __forceinline__ double mul_rounded(double a, double b)
{
#pragma clang fp contract(off)
  return a * b;
}
__device__ __forceinline__ unsigned gstride() { return gridDim.x * blockDim.x; }

// XCD-aware sweep ranges.  Workgroups are dispatched round-robin over the 8
// XCDs (block b runs on XCD b % 8), each with its own L2.  With a plain
// grid-stride loop the y/z neighbours of a block's cells belong to blocks on
// other XCDs and are fetched again from the Infinity Cache / HBM by every XCD.
// Instead the blocks of XCD k sweep one contiguous eighth of the array, so
// neighbour lines stay in that XCD's L2.  Used when the grid is a multiple of
// 8 blocks (host launches round to that); otherwise plain grid-stride.
constexpr unsigned NXCD = 8;
__device__ __forceinline__ bool xcd_on() { return gridDim.x >= NXCD && (gridDim.x % NXCD) == 0; }
__device__ __forceinline__ unsigned xchunk(unsigned n) { return (n + NXCD - 1) / NXCD; }
__device__ __forceinline__ unsigned xbeg(unsigned n)
{
  return xcd_on() ? (blockIdx.x % NXCD) * xchunk(n) + (blockIdx.x / NXCD) * blockDim.x + threadIdx.x : gtid();
}
__device__ __forceinline__ unsigned xend(unsigned n)
{
  if (!xcd_on()) return n;
  const unsigned e = (blockIdx.x % NXCD + 1) * xchunk(n);
  return e < n ? e : n;
}
__device__ __forceinline__ unsigned xstride() { return xcd_on() ? (gridDim.x / NXCD) * blockDim.x : gstride(); }

__device__ __forceinline__ void unflat(const int dims[3], unsigned id, int x[3])
{
  unsigned t = id / (unsigned)dims[0];
  x[0] = (int)(id - t * (unsigned)dims[0]);
  unsigned k = t / (unsigned)dims[1];
  x[1] = (int)(t - k * (unsigned)dims[1]);
  x[2] = (int)k;
}

__device__ __forceinline__ unsigned cidx(const Dev &g, int i, int j, int k)
{
  return (unsigned)i + (unsigned)g.n[0] * ((unsigned)j + (unsigned)g.n[1] * (unsigned)k);
}

__device__ __forceinline__ unsigned fidx(const Dev &g, int d, int i, int j, int k)
{
  return (unsigned)i + (unsigned)g.fd[d][0] * ((unsigned)j + (unsigned)g.fd[d][1] * (unsigned)k);
}

// Stride of a unit step along direction e in a grid of dims.
__device__ __forceinline__ unsigned dstride(const int dims[3], int e)
{
  return e == 0 ? 1u : (e == 1 ? (unsigned)dims[0] : (unsigned)dims[0] * (unsigned)dims[1]);
}

// Sum over a block of TPB threads (wave64 shuffles, then LDS); result valid in thread 0.
__device__ __forceinline__ double block_sum(double v, double *lds)
{
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s += lds[i];
  return s;
}

__device__ __forceinline__ double block_max(double v, double *lds)
{
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) s = fmax(s, lds[i]);
  return s;
}

// Write NQ block partial sums: part[q * MAXB + blockIdx.x].
template <int NQ>
__device__ __forceinline__ void write_partials(const double (&v)[NQ], double *part)
{
  __shared__ double lds[NQ][TPB / 64];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double s = block_sum(v[q], lds[q]);
    if (threadIdx.x == 0) part[q * MAXB + blockIdx.x] = s;
  }
}

// Fixed-order sum of nb partials of quantity q by one block: thread t adds
// partials t, t + blockDim, ... in that order, then the block sum; valid in
// thread 0.  The loads of a chunk of 16 are all issued before the first add
// (indices clamped into the quantity's slots, the ones past nb dropped by a
// select), so a thread waits for memory once per chunk, not once per partial.
constexpr int PCHUNK = 16;
__device__ __forceinline__ double sum_partials(const double *part, int q, int nb)
{
  __shared__ double lds[TPB / 64];
  double s = 0.0;
  const int st = (int)blockDim.x;
  for (int b0 = threadIdx.x; b0 < nb; b0 += PCHUNK * st) {
    double v[PCHUNK];
#pragma unroll
    for (int k = 0; k < PCHUNK; ++k) v[k] = part[q * MAXB + min(b0 + k * st, MAXB - 1)];
#pragma unroll
    for (int k = 0; k < PCHUNK; ++k) s = b0 + k * st < nb ? s + v[k] : s;
  }
  return block_sum(s, lds);
}

__device__ __forceinline__ double max_partials(const double *part, int q, int nb)
{
  __shared__ double lds[TPB / 64];
  double s = 0.0;
  const int st = (int)blockDim.x;
  for (int b0 = threadIdx.x; b0 < nb; b0 += PCHUNK * st) {
    double v[PCHUNK];
#pragma unroll
    for (int k = 0; k < PCHUNK; ++k) v[k] = part[q * MAXB + min(b0 + k * st, MAXB - 1)];
#pragma unroll
    for (int k = 0; k < PCHUNK; ++k) s = b0 + k * st < nb ? fmax(s, v[k]) : s;
  }
  return block_max(s, lds);
}

// In-place Gauss-Jordan inverse of the n x n matrix M (n <= 64, in LDS, row
// stride 65) without pivoting (the matrices are SPD), by a block of
// GJ_TPB threads.  Step k: piv = 1 / M[k][k]; row k is scaled by piv; every other
// element takes M[i][j] - M[i][k] (M[k][j] piv); column k becomes
// -M[i][k] piv and M[k][k] = piv.  Every thread keeps its own elements in
// registers for all steps; only the pivot row and column travel through LDS
// (rowk / colk, 2 x 64 each, double-buffered: the threads that update row and
// column k + 1 in step k publish them for step k + 1), so a step needs one
// barrier.
// A block of 1024 threads: one to four elements per thread, so the few waves
// of this single-block kernel do little work each between barriers.
constexpr int GJ_TPB = 1024;
__device__ __forceinline__ void gauss_jordan_inverse(double (*M)[65], int n, double (*rowk)[64], double (*colk)[64])
{
  constexpr int PER = (64 * 64 + GJ_TPB - 1) / GJ_TPB;
  double v[PER];
  int ei[PER], ej[PER];
  const int nn = n * n;
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int e = min((int)threadIdx.x + m * GJ_TPB, nn - 1);
    ei[m] = e / n;
    ej[m] = e - ei[m] * n;
    v[m] = M[ei[m]][ej[m]];
    if ((int)threadIdx.x + m * GJ_TPB < nn) {
      if (ei[m] == 0) rowk[0][ej[m]] = v[m];
      if (ej[m] == 0) colk[0][ei[m]] = v[m];
    }
  }
  for (int k = 0; k < n; ++k) {
    __syncthreads();
    const double *rk = rowk[k & 1], *ck = colk[k & 1];
    double *rn = rowk[(k + 1) & 1], *cn = colk[(k + 1) & 1];
    const double piv = 1.0 / rk[k];
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      if ((int)threadIdx.x + m * GJ_TPB >= nn) continue;
      const int i = ei[m], j = ej[m];
      double x = v[m];
      if (i == k) x = j == k ? piv : rk[j] * piv;
      else if (j == k) x = -ck[i] * piv;
      else x -= ck[i] * (rk[j] * piv);
      v[m] = x;
      if (i == k + 1) rn[j] = x;
      if (j == k + 1) cn[i] = x;
    }
  }
  __syncthreads();
#pragma unroll
  for (int m = 0; m < PER; ++m)
    if ((int)threadIdx.x + m * GJ_TPB < nn) M[ei[m]][ej[m]] = v[m];
  __syncthreads();
}

// van Leer (1974) correction to the upwind face value: with a = phi_C - phi_U and
// b = phi_D - phi_C the face value is phi_C + a b / (a + b) when a b > 0, else phi_C.
__device__ __forceinline__ double vanleer_corr(double pu, double pc, double pd)
{
  const double a = pc - pu, b = pd - pc;
  return (a * b > 0.0) ? a * b / (a + b) : 0.0;
}

}  // namespace vos
