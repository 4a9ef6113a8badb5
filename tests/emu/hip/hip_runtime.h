// Host stand-in for the HIP runtime header, used only by the CPU emulation of
// the marching kernels (tests/emu/zmarch_emu.cpp).  A kernel becomes a plain
// function; the harness runs it once per (block, thread) with blockIdx and
// threadIdx set, one thread after another.  The kernels' addresses depend only
// on the launch indices and the level dimensions, never on data, so this
// sequential run touches exactly the addresses the device launch touches;
// barriers are no-ops and wave shuffles return their own operand (values are
// not checked, only where they are read and written).
#pragma once
#include <algorithm>
#include <cmath>
#include <cstddef>
#include <cstdint>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __restrict__ __restrict

struct emu_dim3 {
  unsigned x = 0, y = 0, z = 0;
};
extern emu_dim3 threadIdx, blockIdx, blockDim, gridDim;

inline void __syncthreads() {}
template <typename T>
inline T __shfl_down(T v, unsigned, int) { return v; }

inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
using std::fmax;
using std::sqrt;
