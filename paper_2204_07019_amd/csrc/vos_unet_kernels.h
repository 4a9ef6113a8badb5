// vos_unet_kernels.h -- BF16 MFMA kernels of the pressure warm-start U-Net
// (3-D, 3x3x3 convolutions, NDHWC activations, FP32 accumulation).
//
// The convolutions are dense contractions, so they run on the matrix cores:
// v_mfma_f32_16x16x16bf16_1k, one wave computing a 16-voxel x 16-channel tile
// per instruction.  Operand layout of that instruction (wave64), used
// throughout:
//   A (16 x 16, M x K): lane l holds A[l % 16][4 (l / 16) + j], j = 0..3
//   B (16 x 16, K x N): lane l holds B[4 (l / 16) + j][l % 16]
//   D (16 x 16, M x N): lane l holds D[4 (l / 16) + i][l % 16], i = 0..3
// Forward: M = 16 consecutive voxels along x, N = output channels, K = input
// channels of one tap (the 27 taps accumulate into the same tile).  The data
// gradient is the same kernel on the output gradient with flipped, transposed
// weights.  The weight gradient contracts over voxels (M = input channels,
// N = output channels, K = voxels) with a deterministic split-K reduction.
#pragma once
#include <hip/hip_runtime.h>

namespace vosnet {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int CTPB = 256;         // 4 waves per block
constexpr int WG_CHUNKS = 64;     // weight-gradient partial buffer: WG_CHUNKS x 27 x max(ci co) floats

// Round-to-nearest-even FP32 -> BF16 (NaN kept quiet).
__device__ __forceinline__ unsigned short f2bf(float f)
{
  unsigned u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return 0x7fc0;
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float bf2f(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

struct Vol {   // one NDHWC activation tensor (a channel slice of a buffer)
  unsigned short *p;
  int ctot;    // channels per voxel in the buffer
  int coff;    // first channel of the slice
};

// Convolution, forward and data gradient: y[v][co] = sum over the 27 taps
// (in order) and the input channels (chunks of 16, in order) of
// x[v + off(tap)][ci] w[tap][co][ci] (+ bias[co]), zero padding, FP32
// accumulation; optional ReLU; optional mask (y = 0 where m[v][co] <= 0);
// output as BF16 into a channel slice, or as FP32 (y32, dense Cout channels).
// The data gradient is this kernel on the output gradient with the flipped,
// transposed weights.  A block of 4 waves owns 64 x-voxels (4 matrix tiles of 16) x 4 rows (wave w: row
// 4 by + w) at one z; per chunk of 16 input channels the 3 x 6 x 66 halo of
// the input is staged in LDS once, as [z][y][channel quad][x] of 4 BF16 each,
// together with the chunk's weight fragments of all 27 taps ([tap][tile][lane],
// so no global load sits inside the tap loop); a wave reads its A and B
// fragments from LDS, and each weight fragment is reused for the 4 matrix
// tiles.  Grid (ceil(W / 64), ceil(H / 4), N * D).  Requires Cin % 16 == 0.
constexpr int KT_X = 64, KT_Y = 4, KH_X = KT_X + 2, KH_Y = KT_Y + 2;

template <int NT>
__global__ void __launch_bounds__(CTPB) k_conv3d_tile(Vol x, int Cin, const unsigned short *__restrict__ w,
                                                      const float *__restrict__ bias, Vol y, float *__restrict__ y32,
                                                      int D, int H, int W, int relu, Vol mask)
{
  constexpr int Cout = NT * 16;
  __shared__ __align__(16) bf16x4 tile[3][KH_Y][4][KH_X];
  __shared__ __align__(16) bf16x4 wl[27][NT][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int x0 = blockIdx.x * KT_X, y0 = blockIdx.y * KT_Y;
  const int z = blockIdx.z % D, n = blockIdx.z / D;
  const int yy = y0 + wv;
  f32x4 acc[4][NT];
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int t = 0; t < NT; ++t) acc[mt][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nchunk = Cin >> 4;
  // staging: every load of a thread is issued before any is waited for (addresses
  // clamped into the tensor, zero padding selected afterwards)
  constexpr int NX = 3 * KH_Y * KH_X * 4, PX = (NX + CTPB - 1) / CTPB;
  constexpr int NWF = 27 * NT * 64, PW = (NWF + CTPB - 1) / CTPB;
  for (int cc = 0; cc < nchunk; ++cc) {
    bf16x4 xv[PX], wv4[PW];
#pragma unroll
    for (int i = 0; i < PX; ++i) {
      const int e = min((int)threadIdx.x + i * CTPB, NX - 1);
      const int q = e & 3, vox = e >> 2;
      const int hx = vox % KH_X, hy = (vox / KH_X) % KH_Y, hz = vox / (KH_X * KH_Y);
      const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z + hz - 1;
      const int cx = min(max(gx, 0), W - 1), cy = min(max(gy, 0), H - 1), cz = min(max(gz, 0), D - 1);
      const size_t gv = (((size_t)n * D + cz) * H + cy) * W + cx;
      const bf16x4 v = *(const bf16x4 *)(x.p + gv * x.ctot + x.coff + cc * 16 + q * 4);
      const bool in = gx >= 0 && gx < W && gy >= 0 && gy < H && gz >= 0 && gz < D;
      xv[i] = in ? v : bf16x4{0, 0, 0, 0};
    }
    // B fragment of lane l for tap and output tile t: w[tap][t 16 + l % 16][16 cc + 4 (l / 16) .. + 3]
#pragma unroll
    for (int i = 0; i < PW; ++i) {
      const int e = min((int)threadIdx.x + i * CTPB, NWF - 1);
      const int ln = e & 63, t = (e >> 6) % NT, tap = (e >> 6) / NT;
      wv4[i] = *(const bf16x4 *)(w + (size_t)tap * Cout * Cin + (size_t)(t * 16 + (ln & 15)) * Cin + cc * 16 +
                                 (ln >> 4) * 4);
    }
    __syncthreads();   // the previous chunk's tile has been consumed
#pragma unroll
    for (int i = 0; i < PX; ++i) {
      const int e = (int)threadIdx.x + i * CTPB;
      if (e >= NX) break;
      const int q = e & 3, vox = e >> 2;
      tile[vox / (KH_X * KH_Y)][(vox / KH_X) % KH_Y][q][vox % KH_X] = xv[i];
    }
#pragma unroll
    for (int i = 0; i < PW; ++i) {
      const int e = (int)threadIdx.x + i * CTPB;
      if (e >= NWF) break;
      wl[(e >> 6) / NT][(e >> 6) % NT][e & 63] = wv4[i];
    }
    __syncthreads();
    if (yy < H) {
      for (int tap = 0; tap < 27; ++tap) {
        const int dz = tap / 9, dy = (tap / 3) % 3, dx = tap % 3;
        bf16x4 b[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) b[t] = wl[tap][t][lane];
#pragma unroll
        for (int mt = 0; mt < 4; ++mt) {
          const bf16x4 a = tile[dz][wv + dy][kq][mt * 16 + m + dx];
#pragma unroll
          for (int t = 0; t < NT; ++t) acc[mt][t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b[t], acc[mt][t], 0, 0, 0);
        }
      }
    }
  }
  if (yy >= H) return;
#pragma unroll
  for (int mt = 0; mt < 4; ++mt)
#pragma unroll
    for (int t = 0; t < NT; ++t) {
      const int co = t * 16 + m;
      const float bco = bias ? bias[co] : 0.f;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int xv = x0 + mt * 16 + kq * 4 + i;
        if (xv >= W) continue;
        const size_t vox = (((size_t)n * D + z) * H + yy) * W + xv;
        float v = acc[mt][t][i] + bco;
        if (relu) v = v > 0.f ? v : 0.f;
        if (mask.p && !(bf2f(mask.p[vox * mask.ctot + mask.coff + co]) > 0.f)) v = 0.f;
        if (y32) y32[vox * Cout + co] = v;
        else y.p[vox * y.ctot + y.coff + co] = f2bf(v);
      }
    }
}

// Tiled weight gradient.  Block (group g, channel-tile pair) loops over the
// spatial tiles g, g + groups, ... (64 x-voxels x 4 rows at one z; wave w owns
// row w) and accumulates, for all 27 taps, dW[tap][ci][co] += x[v + off][ci]
// dy[v][co] over the tile's voxels (K = voxels, 16 per matrix step).  Per
// tile the input halo (16 channels, 3 x 6 x 66) is staged channel-major in
// LDS with x contiguous, so one aligned 8-byte read gives 4 consecutive
// voxels; the x-shifted operands of the three dx taps are formed from it and
// the two edge voxels by 64-bit shifts.  The 4 waves' sums are added in fixed
// order and written as partial g: part[((g * 27 + tap) * Cin + ci) * Cout + co].
constexpr int WX_P = 72;   // LDS row: halo x index hx stored at hx + 3 (interior quads 8-byte aligned)

__global__ void __launch_bounds__(CTPB) k_conv3d_wgrad_tile(Vol x, int Cin, Vol dy, int Cout, int N, int D, int H,
                                                           int W, int groups, float *__restrict__ part)
{
  __shared__ __align__(16) unsigned short xt[16][3][KH_Y][WX_P];   // 41472 B; rows of 144 B
  __shared__ __align__(16) unsigned short dt[16][KT_Y][KT_X];      // 8192 B; rows of 128 B
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int m = lane & 15, kq = lane >> 4;
  const int ntc = Cout >> 4;
  const int cit = blockIdx.y / ntc, cot = blockIdx.y % ntc;
  const int gx = (W + KT_X - 1) / KT_X, gy = (H + KT_Y - 1) / KT_Y;
  const long long ntiles = (long long)gx * gy * D * N;
  f32x4 acc[27];
#pragma unroll
  for (int t = 0; t < 27; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  // staging of a tile: every load is issued before any is waited for (addresses clamped
  // into the tensors, zero padding selected afterwards); the next tile's loads are in
  // flight while the current tile is contracted
  constexpr int NX = 3 * KH_Y * KH_X * 4, PX = (NX + CTPB - 1) / CTPB;
  constexpr int ND = KT_Y * KT_X * 4, PD = (ND + CTPB - 1) / CTPB;
  bf16x4 xv[PX], dv[PD];
  auto load = [&](long long tile) {
    const int tx = (int)(tile % gx), ty = (int)((tile / gx) % gy);
    const int z = (int)((tile / ((long long)gx * gy)) % D), n = (int)(tile / ((long long)gx * gy * D));
    const int x0 = tx * KT_X, y0 = ty * KT_Y;
#pragma unroll
    for (int i = 0; i < PX; ++i) {
      const int e = min((int)threadIdx.x + i * CTPB, NX - 1);
      const int q = e & 3, vox = e >> 2;
      const int hx = vox % KH_X, hy = (vox / KH_X) % KH_Y, hz = vox / (KH_X * KH_Y);
      const int ix = x0 + hx - 1, iy = y0 + hy - 1, iz = z + hz - 1;
      const int cx = min(max(ix, 0), W - 1), cy = min(max(iy, 0), H - 1), cz = min(max(iz, 0), D - 1);
      const size_t gv = (((size_t)n * D + cz) * H + cy) * W + cx;
      const bf16x4 v = *(const bf16x4 *)(x.p + gv * x.ctot + x.coff + cit * 16 + q * 4);
      xv[i] = (ix >= 0 && ix < W && iy >= 0 && iy < H && iz >= 0 && iz < D) ? v : bf16x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int i = 0; i < PD; ++i) {
      const int e = min((int)threadIdx.x + i * CTPB, ND - 1);
      const int q = e & 3, vox = e >> 2;
      const int ix = x0 + vox % KT_X, iy = y0 + vox / KT_X;
      const size_t gv = (((size_t)n * D + z) * H + min(iy, H - 1)) * W + min(ix, W - 1);
      const bf16x4 v = *(const bf16x4 *)(dy.p + gv * dy.ctot + dy.coff + cot * 16 + q * 4);
      dv[i] = (ix < W && iy < H) ? v : bf16x4{0, 0, 0, 0};
    }
  };
  if (blockIdx.x < ntiles) load(blockIdx.x);
  for (long long tile = blockIdx.x; tile < ntiles; tile += groups) {
    __syncthreads();   // previous tile consumed
#pragma unroll
    for (int i = 0; i < PX; ++i) {
      const int e = (int)threadIdx.x + i * CTPB;
      if (e >= NX) break;
      const int q = e & 3, vox = e >> 2;
      const int hx = vox % KH_X, hy = (vox / KH_X) % KH_Y, hz = vox / (KH_X * KH_Y);
#pragma unroll
      for (int j = 0; j < 4; ++j) xt[q * 4 + j][hz][hy][hx + 3] = (unsigned short)xv[i][j];
    }
#pragma unroll
    for (int i = 0; i < PD; ++i) {
      const int e = (int)threadIdx.x + i * CTPB;
      if (e >= ND) break;
      const int q = e & 3, vox = e >> 2;
#pragma unroll
      for (int j = 0; j < 4; ++j) dt[q * 4 + j][vox / KT_X][vox % KT_X] = (unsigned short)dv[i][j];
    }
    __syncthreads();
    if (tile + groups < ntiles) load(tile + groups);
    for (int g16 = 0; g16 < KT_X / 16; ++g16) {
      const int xq = g16 * 16 + kq * 4;   // first voxel of this lane's quad (interior x index)
      const bf16x4 b = *(const bf16x4 *)&dt[m][wv][xq];
#pragma unroll
      for (int c = 0; c < 9; ++c) {
        const int dz = c / 3, dyy = c % 3;
        const unsigned short *row = &xt[m][dz][wv + dyy][0];
        const unsigned long long Q = *(const unsigned long long *)(row + xq + 4);
        const unsigned long long eL = row[xq + 3], eR = row[xq + 8];
        const unsigned long long A0 = (Q << 16) | eL, A2 = (Q >> 16) | (eR << 48);
        bf16x4 a0, a1, a2;
        __builtin_memcpy(&a0, &A0, 8);
        __builtin_memcpy(&a1, &Q, 8);
        __builtin_memcpy(&a2, &A2, 8);
        acc[c * 3 + 0] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a0, b, acc[c * 3 + 0], 0, 0, 0);
        acc[c * 3 + 1] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a1, b, acc[c * 3 + 1], 0, 0, 0);
        acc[c * 3 + 2] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a2, b, acc[c * 3 + 2], 0, 0, 0);
      }
    }
  }
  // add the 4 waves (fixed order) and write this group's partial
  __syncthreads();
  float *red = reinterpret_cast<float *>(&xt[0][0][0][0]);   // 4 x 256 floats
#pragma unroll
  for (int tap = 0; tap < 27; ++tap) {
#pragma unroll
    for (int i = 0; i < 4; ++i) red[wv * 256 + (kq * 4 + i) * 16 + m] = acc[tap][i];
    __syncthreads();
    const int e = threadIdx.x;   // 16 ci x 16 co
    const float sum = red[e] + red[256 + e] + red[512 + e] + red[768 + e];
    const int ci = cit * 16 + e / 16, co = cot * 16 + e % 16;
    part[(((size_t)blockIdx.x * 27 + tap) * Cin + ci) * Cout + co] = sum;
    __syncthreads();
  }
}

// dW[tap][ci][co] = sum over the `chunks` partials (fixed order: lane l of 8
// sums chunks l, l + 8, ... in turn, then the 8 lane sums are added in lane
// order).  Block CTPB = 32 weights x 8 lanes.
__global__ void __launch_bounds__(CTPB) k_wgrad_reduce(const float *__restrict__ part, int n, int chunks,
                                                       float *__restrict__ dw)
{
  __shared__ float red[8][32];
  const int wl = threadIdx.x & 31, l = threadIdx.x >> 5;
  const int i = blockIdx.x * 32 + wl;
  float s = 0.f;
  if (i < n)
    for (int c = l; c < chunks; c += 8) s += part[(size_t)c * n + i];
  red[l][wl] = s;
  __syncthreads();
  if (l == 0 && i < n) {
    float t = 0.f;
    for (int k = 0; k < 8; ++k) t += red[k][wl];
    dw[i] = t;
  }
}

// Bias gradient partials: per block, sum of dy over its voxels, per channel.
// Grid: nblk blocks over V voxels; block 256 = C channels x (256/C) voxel lanes.
__global__ void k_bias_grad_part(Vol dy, int C, size_t V, float *__restrict__ part)
{
  __shared__ float red[256];
  const int c = threadIdx.x % C, lane = threadIdx.x / C, lanes = CTPB / C;
  float s = 0.f;
  if (lane < lanes)
    for (size_t v = (size_t)blockIdx.x * lanes + lane; v < V; v += (size_t)gridDim.x * lanes)
      s += bf2f(dy.p[v * dy.ctot + dy.coff + c]);
  red[threadIdx.x] = s;
  __syncthreads();
  if (lane == 0) {
    float t = 0.f;
    for (int l = 0; l < lanes; ++l) t += red[l * C + c];
    part[(size_t)blockIdx.x * C + c] = t;
  }
}

// db[c] = sum over the nblk partials (fixed order): one block of CTPB threads,
// each thread sums a strided subset of the partials of every channel, then a
// tree over the threads.  C <= 64.
__global__ void __launch_bounds__(CTPB) k_bias_grad_final(const float *__restrict__ part, int C, int nblk,
                                                          float *__restrict__ db)
{
  __shared__ float red[CTPB][17];
  for (int c0 = 0; c0 < C; c0 += 16) {
    const int cn = C - c0 < 16 ? C - c0 : 16;
    float acc[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) acc[k] = 0.f;
    for (int b = threadIdx.x; b < nblk; b += CTPB)
#pragma unroll
      for (int k = 0; k < 16; ++k)
        if (k < cn) acc[k] += part[(size_t)b * C + c0 + k];
#pragma unroll
    for (int k = 0; k < 16; ++k) red[threadIdx.x][k] = acc[k];
    __syncthreads();
    for (int o = CTPB / 2; o > 0; o >>= 1) {
      if (threadIdx.x < o)
        for (int k = 0; k < cn; ++k) red[threadIdx.x][k] += red[threadIdx.x + o][k];
      __syncthreads();
    }
    if (threadIdx.x < cn) db[c0 + threadIdx.x] = red[0][threadIdx.x];
    __syncthreads();
  }
}

// 2x2x2 average pooling (fine dims D, H, W even).
__global__ void k_pool_fwd(Vol x, int C, Vol y, int N, int D, int H, int W)
{
  const int Dc = D / 2, Hc = H / 2, Wc = W / 2;
  const size_t total = (size_t)N * Dc * Hc * Wc * C;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    size_t v = i / C;
    const int xc = (int)(v % Wc), yc = (int)((v / Wc) % Hc), zc = (int)((v / ((size_t)Wc * Hc)) % Dc);
    const int n = (int)(v / ((size_t)Wc * Hc * Dc));
    float s = 0.f;
    for (int a = 0; a < 8; ++a) {
      const size_t vf = (((size_t)n * D + 2 * zc + (a >> 2)) * H + 2 * yc + ((a >> 1) & 1)) * W + 2 * xc + (a & 1);
      s += bf2f(x.p[vf * x.ctot + x.coff + c]);
    }
    y.p[v * y.ctot + y.coff + c] = f2bf(0.125f * s);
  }
}

// Gradient of the average pool, optionally added to an existing gradient slice
// and masked by (m > 0): g[f] = (add ? g[f] : 0) + mask(f) * dy[parent] / 8.
// One thread handles 8 channels (C, ctot and coff are multiples of 8).
__global__ void k_pool_bwd(Vol dy, int C, Vol g, int N, int D, int H, int W, int add, Vol mask)
{
  const int C8 = C / 8;
  const size_t total = (size_t)N * D * H * W * C8;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C8) * 8;
    const size_t v = i / C8;
    const int xx = (int)(v % W), yy = (int)((v / W) % H), zz = (int)((v / ((size_t)W * H)) % D);
    const int n = (int)(v / ((size_t)W * H * D));
    const size_t vc = (((size_t)n * (D / 2) + zz / 2) * (H / 2) + yy / 2) * (W / 2) + xx / 2;
    const uint4 dv = *(const uint4 *)(dy.p + vc * dy.ctot + dy.coff + c);
    const unsigned short *d8 = reinterpret_cast<const unsigned short *>(&dv);
    uint4 mv = uint4{0, 0, 0, 0}, gv = uint4{0, 0, 0, 0};
    if (mask.p) mv = *(const uint4 *)(mask.p + v * mask.ctot + mask.coff + c);
    unsigned short *gp = g.p + v * g.ctot + g.coff + c;
    if (add) gv = *(const uint4 *)gp;
    const unsigned short *m8 = reinterpret_cast<const unsigned short *>(&mv);
    const unsigned short *g8 = reinterpret_cast<const unsigned short *>(&gv);
    uint4 ov;
    unsigned short *o8 = reinterpret_cast<unsigned short *>(&ov);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      float d = 0.125f * bf2f(d8[k]);
      if (mask.p && !(bf2f(m8[k]) > 0.f)) d = 0.f;
      o8[k] = f2bf(add ? bf2f(g8[k]) + d : d);
    }
    *(uint4 *)gp = ov;
  }
}

// Nearest-neighbour 2x upsampling into a channel slice: y[f] = x[parent(f)].
// One thread moves 8 channels (16 bytes): C, ctot and coff are multiples of 8.
__global__ void k_up_fwd(Vol x, int C, Vol y, int N, int D, int H, int W)
{
  const int C8 = C / 8;
  const size_t total = (size_t)N * D * H * W * C8;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C8) * 8;
    const size_t v = i / C8;
    const int xx = (int)(v % W), yy = (int)((v / W) % H), zz = (int)((v / ((size_t)W * H)) % D);
    const int n = (int)(v / ((size_t)W * H * D));
    const size_t vc = (((size_t)n * (D / 2) + zz / 2) * (H / 2) + yy / 2) * (W / 2) + xx / 2;
    *(uint4 *)(y.p + v * y.ctot + y.coff + c) = *(const uint4 *)(x.p + vc * x.ctot + x.coff + c);
  }
}

// Gradient of the upsampling: g[parent] = sum of the 8 children's gradients.
__global__ void k_up_bwd(Vol dy, int C, Vol g, int N, int D, int H, int W)
{
  const int Dc = D / 2, Hc = H / 2, Wc = W / 2;
  const size_t total = (size_t)N * Dc * Hc * Wc * C;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % C);
    const size_t v = i / C;
    const int xc = (int)(v % Wc), yc = (int)((v / Wc) % Hc), zc = (int)((v / ((size_t)Wc * Hc)) % Dc);
    const int n = (int)(v / ((size_t)Wc * Hc * Dc));
    float s = 0.f;
    for (int a = 0; a < 8; ++a) {
      const size_t vf = (((size_t)n * D + 2 * zc + (a >> 2)) * H + 2 * yc + ((a >> 1) & 1)) * W + 2 * xc + (a & 1);
      s += bf2f(dy.p[vf * dy.ctot + dy.coff + c]);
    }
    g.p[v * g.ctot + g.coff + c] = f2bf(s);
  }
}

// FP32 NDHWC input with cin real channels -> BF16 with 16 channels (zero padded).
__global__ void k_pack_input(const float *__restrict__ xin, int cin, size_t V, Vol y)
{
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < V * 16; i += (size_t)gridDim.x * blockDim.x) {
    const int c = (int)(i % 16);
    const size_t v = i / 16;
    y.p[v * y.ctot + y.coff + c] = c < cin ? f2bf(xin[v * cin + c]) : (unsigned short)0;
  }
}

// Head (1x1x1, 16 -> 1, FP32): out[v] = sum_c w[c] x[v][c] + b.
__global__ void k_head_fwd(Vol x, const float *__restrict__ w, const float *__restrict__ b, size_t V,
                           float *__restrict__ out)
{
  for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < V; v += (size_t)gridDim.x * blockDim.x) {
    float s = b[0];
    for (int c = 0; c < 16; ++c) s += w[c] * bf2f(x.p[v * x.ctot + x.coff + c]);
    out[v] = s;
  }
}

// MSE: dy = 2 (y - t) / V (FP32), and per-block partial sums of (y - t)^2.
__global__ void k_mse(const float *__restrict__ y, const float *__restrict__ t, size_t V, float *__restrict__ dy,
                      double *__restrict__ part)
{
  __shared__ double red[CTPB];
  double s = 0.0;
  for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < V; v += (size_t)gridDim.x * blockDim.x) {
    const float d = y[v] - t[v];
    dy[v] = 2.f * d / (float)V;
    s += (double)d * d;
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = CTPB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Head backward: gx[v][c] = mask(v,c) * w[c] dy[v] (BF16); partials of
// dw[c] = sum_v x[v][c] dy[v] and db = sum_v dy[v] per block (17 values).
__global__ void k_head_bwd(Vol x, const float *__restrict__ w, const float *__restrict__ dy, size_t V, Vol gx,
                           float *__restrict__ part)
{
  __shared__ float red[17][CTPB];
  float s[17];
  for (int k = 0; k < 17; ++k) s[k] = 0.f;
  for (size_t v = blockIdx.x * (size_t)blockDim.x + threadIdx.x; v < V; v += (size_t)gridDim.x * blockDim.x) {
    const float d = dy[v];
    for (int c = 0; c < 16; ++c) {
      const float xv = bf2f(x.p[v * x.ctot + x.coff + c]);
      s[c] += xv * d;
      gx.p[v * gx.ctot + gx.coff + c] = f2bf(xv > 0.f ? w[c] * d : 0.f);
    }
    s[16] += d;
  }
  for (int k = 0; k < 17; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  if (threadIdx.x < 17) {
    float t = 0.f;
    for (int i = 0; i < CTPB; ++i) t += red[threadIdx.x][i];
    part[(size_t)blockIdx.x * 17 + threadIdx.x] = t;
  }
}

// Master FP32 weights [tap][ci][co] -> forward layout [tap][co][ci] and
// data-gradient layout [26 - tap][ci][co] as BF16 (the latter is the forward
// layout of the transposed, flipped convolution; skipped when wd is null).
__global__ void k_weights_to_bf16(const float *__restrict__ wm, int Cin, int Cout, unsigned short *__restrict__ wf,
                                  unsigned short *__restrict__ wd)
{
  const int n = 27 * Cin * Cout;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int co = i % Cout, ci = (i / Cout) % Cin, tap = i / (Cout * Cin);
    const unsigned short h = f2bf(wm[i]);
    wf[((size_t)tap * Cout + co) * Cin + ci] = h;
    if (wd) wd[((size_t)(26 - tap) * Cin + ci) * Cout + co] = h;
  }
}

// Adam (Kingma & Ba 2015) on FP32 master parameters.
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ g, float *__restrict__ m, float *__restrict__ v,
                       int n, float lr, float b1, float b2, float eps, float c1, float c2)
{
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

}  // namespace vosnet

namespace vosnet {
// Fixed-order sum of n double partials by one block of CTPB threads.
__global__ void k_sum_double(const double *__restrict__ part, int n, double *__restrict__ out)
{
  __shared__ double red[CTPB];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += CTPB) s += part[i];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int o = CTPB / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[0] = red[0];
}
}  // namespace vosnet
