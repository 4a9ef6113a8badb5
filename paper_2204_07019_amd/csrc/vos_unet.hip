// vos_unet.hip -- host side of the warm-start U-Net (include/vos_unet.h):
// workspace layout, forward, backward, Adam.  Every arithmetic step runs in
// the kernels of vos_unet_kernels.h on the network's stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "vos_internal.h"
#include "vos_unet_kernels.h"

using namespace vosnet;
using vosint::fail;

namespace {

#define UN_TRY(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(VOS_ERR_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));        \
  } while (0)

constexpr int NL = 10;
struct LayerDef { int ci, co, level; };
constexpr LayerDef LAY[NL] = {{16, 16, 0}, {16, 16, 0}, {16, 32, 1}, {32, 32, 1}, {32, 64, 2},
                              {64, 64, 2}, {96, 32, 1}, {32, 32, 1}, {48, 16, 0}, {16, 16, 0}};
enum { E0A, E0B, E1A, E1B, BA, BB, D1A, D1B, D0A, D0B };

size_t wsize(int l) { return (size_t)27 * LAY[l].ci * LAY[l].co; }
size_t layer_off(int l)
{
  size_t o = 0;
  for (int k = 0; k < l; ++k) o += wsize(k) + LAY[k].co;
  return o;
}
size_t head_off() { return layer_off(NL); }
// Largest ci * co of any layer: the weight-gradient partials hold
// WG_CHUNKS * 27 * this many floats.
constexpr size_t max_cico()
{
  size_t m = 0;
  for (int l = 0; l < NL; ++l) m = (size_t)LAY[l].ci * LAY[l].co > m ? (size_t)LAY[l].ci * LAY[l].co : m;
  return m;
}
constexpr size_t WPART_FLOATS = (size_t)WG_CHUNKS * 27 * max_cico();
static_assert(max_cico() == 64 * 64, "layer table changed: check the partial-sum buffer");
size_t n_params() { return head_off() + 17; }

constexpr int NB_BIAS = 1024;   // partial-sum blocks of the bias / head gradients and the loss
constexpr size_t ALIGN = 256;

int eblocks(size_t n)
{
  size_t b = (n + CTPB - 1) / CTPB;
  return (int)(b < 1 ? 1 : (b > 8192 ? 8192 : b));
}

}  // namespace

struct vos_unet {
  int N, D, H, W, cin, train;
  int dd[3][3];     // (D, H, W) per level
  size_t V[3];      // voxels (all batch entries) per level
  hipStream_t stream;
  float *theta, *grad, *m, *v;
  unsigned short *wf[NL], *wd[NL];
  float *wpart, *bpart, *hpart;
  double *lpart, *lsum;
  float *xin, *yout, *dy;
  unsigned short *X0, *A0, *C0, *P0, *A1, *C1, *P1, *A2, *B2, *D1, *E1, *D0, *E0;
  unsigned short *gE0, *gD0, *gC0, *gE1, *gD1, *gC1, *gB2, *gA2, *gP1, *gA1, *gP0, *gA0;
  double *host;     // pinned: the loss read back
  int t;
};

namespace {

struct Carve {
  char *base;
  size_t off = 0;
  template <typename T>
  T *take(size_t n)
  {
    T *p = base ? (T *)(base + off) : nullptr;
    off += (n * sizeof(T) + ALIGN - 1) / ALIGN * ALIGN;
    return p;
  }
};

// Assign every device array of `u` from `base` (nullptr: size only).
size_t layout(vos_unet *u, char *base)
{
  Carve c{base};
  typedef unsigned short bf;
  const size_t P = n_params();
  const size_t V0 = u->V[0], V1 = u->V[1], V2 = u->V[2];
  u->theta = c.take<float>(P);
  for (int l = 0; l < NL; ++l) u->wf[l] = c.take<bf>(wsize(l));
  u->xin = c.take<float>(V0 * u->cin);
  u->yout = c.take<float>(V0);
  u->X0 = c.take<bf>(V0 * 16);
  u->A0 = c.take<bf>(V0 * 16);
  u->C0 = c.take<bf>(V0 * 48);
  u->D0 = c.take<bf>(V0 * 16);
  u->E0 = c.take<bf>(V0 * 16);
  u->P0 = c.take<bf>(V1 * 16);
  u->A1 = c.take<bf>(V1 * 32);
  u->C1 = c.take<bf>(V1 * 96);
  u->D1 = c.take<bf>(V1 * 32);
  u->E1 = c.take<bf>(V1 * 32);
  u->P1 = c.take<bf>(V2 * 32);
  u->A2 = c.take<bf>(V2 * 64);
  u->B2 = c.take<bf>(V2 * 64);
  if (u->train) {
    u->grad = c.take<float>(P);
    u->m = c.take<float>(P);
    u->v = c.take<float>(P);
    for (int l = 0; l < NL; ++l) u->wd[l] = c.take<bf>(wsize(l));
    u->wpart = c.take<float>(WPART_FLOATS);
    u->bpart = c.take<float>((size_t)NB_BIAS * 64);
    u->hpart = c.take<float>((size_t)NB_BIAS * 17);
    u->lpart = c.take<double>(NB_BIAS);
    u->lsum = c.take<double>(1);
    u->dy = c.take<float>(V0);
    u->gE0 = c.take<bf>(V0 * 16);
    u->gD0 = c.take<bf>(V0 * 16);
    u->gC0 = c.take<bf>(V0 * 48);
    u->gA0 = c.take<bf>(V0 * 16);
    u->gE1 = c.take<bf>(V1 * 32);
    u->gD1 = c.take<bf>(V1 * 32);
    u->gC1 = c.take<bf>(V1 * 96);
    u->gA1 = c.take<bf>(V1 * 32);
    u->gP0 = c.take<bf>(V1 * 16);
    u->gB2 = c.take<bf>(V2 * 64);
    u->gA2 = c.take<bf>(V2 * 64);
    u->gP1 = c.take<bf>(V2 * 32);
  } else {
    u->grad = u->m = u->v = nullptr;
    for (int l = 0; l < NL; ++l) u->wd[l] = nullptr;
  }
  return c.off;
}

vos_status check_shape(const vos_unet_shape *s)
{
  if (!s) return fail(VOS_ERR_ARG, "shape is NULL");
  if (s->batch < 1 || s->nz < 4 || s->ny < 4 || s->nx < 64)
    return fail(VOS_ERR_ARG, "U-Net shape needs batch >= 1, nz >= 4, ny >= 4, nx >= 64");
  if (s->nx % 64 || s->ny % 4 || s->nz % 4)
    return fail(VOS_ERR_ARG, "U-Net shape needs nx % 64 == 0, ny % 4 == 0, nz % 4 == 0");
  if (s->cin < 1 || s->cin > 16) return fail(VOS_ERR_ARG, "U-Net input channels must be 1..16");
  if (s->ny > 65535 || (long long)s->batch * s->nz > 65535)
    return fail(VOS_ERR_ARG, "U-Net shape exceeds the launch grid (ny <= 65535, batch*nz <= 65535)");
  return VOS_OK;
}

void init_dims(vos_unet *u, const vos_unet_shape *s)
{
  u->N = s->batch;
  u->D = s->nz;
  u->H = s->ny;
  u->W = s->nx;
  u->cin = s->cin;
  u->train = s->train ? 1 : 0;
  for (int l = 0; l < 3; ++l) {
    u->dd[l][0] = s->nz >> l;
    u->dd[l][1] = s->ny >> l;
    u->dd[l][2] = s->nx >> l;
    u->V[l] = (size_t)s->batch * u->dd[l][0] * u->dd[l][1] * u->dd[l][2];
  }
}

inline Vol vol(unsigned short *p, int ctot, int coff = 0) { return Vol{p, ctot, coff}; }
const Vol NOMASK = {nullptr, 0, 0};

void conv(hipStream_t st, Vol x, int Cin, const unsigned short *w, const float *bias, Vol y, float *y32, int Cout,
          int N, const int *d, int relu, Vol mask)
{
  const dim3 grid((d[2] + KT_X - 1) / KT_X, (d[1] + KT_Y - 1) / KT_Y, N * d[0]);
  switch (Cout / 16) {
    case 1: k_conv3d_tile<1><<<grid, CTPB, 0, st>>>(x, Cin, w, bias, y, y32, d[0], d[1], d[2], relu, mask); break;
    case 2: k_conv3d_tile<2><<<grid, CTPB, 0, st>>>(x, Cin, w, bias, y, y32, d[0], d[1], d[2], relu, mask); break;
    case 3: k_conv3d_tile<3><<<grid, CTPB, 0, st>>>(x, Cin, w, bias, y, y32, d[0], d[1], d[2], relu, mask); break;
    case 4: k_conv3d_tile<4><<<grid, CTPB, 0, st>>>(x, Cin, w, bias, y, y32, d[0], d[1], d[2], relu, mask); break;
    case 6: k_conv3d_tile<6><<<grid, CTPB, 0, st>>>(x, Cin, w, bias, y, y32, d[0], d[1], d[2], relu, mask); break;
    default: break;   // unreachable: the layer table holds 16, 32, 48, 64 and 96
  }
}

void layer_fwd(vos_unet *u, hipStream_t st, int l, Vol in, Vol out)
{
  const int lv = LAY[l].level;
  conv(st, in, LAY[l].ci, u->wf[l], u->theta + layer_off(l) + wsize(l), out, nullptr, LAY[l].co, u->N, u->dd[lv], 1,
       NOMASK);
}

// Gradients of layer l's weights and bias from the gradient of its
// pre-activation `gout`; if gin.p, also the gradient with respect to its
// input (masked by `mask` > 0 when mask.p).
void layer_bwd(vos_unet *u, hipStream_t st, int l, Vol in, Vol gout, Vol gin, Vol mask)
{
  const int lv = LAY[l].level, ci = LAY[l].ci, co = LAY[l].co;
  const int *d = u->dd[lv];
  const int tiles = (ci / 16) * (co / 16);
  // split-K groups: at most 256 (and what the partial buffer holds for this layer)
  const size_t nw = wsize(l);
  const int groups = (int)std::min<size_t>(256, WPART_FLOATS / nw);
  k_conv3d_wgrad_tile<<<dim3(groups, tiles), CTPB, 0, st>>>(in, ci, gout, co, u->N, d[0], d[1], d[2], groups,
                                                             u->wpart);
  float *g = u->grad + layer_off(l);
  k_wgrad_reduce<<<(unsigned)((nw + 31) / 32), CTPB, 0, st>>>(u->wpart, (int)nw, groups, g);
  k_bias_grad_part<<<NB_BIAS, CTPB, 0, st>>>(gout, co, u->V[lv], u->bpart);
  k_bias_grad_final<<<1, CTPB, 0, st>>>(u->bpart, co, NB_BIAS, g + nw);
  if (gin.p) conv(st, gout, co, u->wd[l], nullptr, gin, nullptr, ci, u->N, d, 0, mask);
}

void forward(vos_unet *u, hipStream_t st, const float *x, float *y)
{
  const int N = u->N;
  const int *d0 = u->dd[0], *d1 = u->dd[1];
  k_pack_input<<<eblocks(u->V[0] * 16), CTPB, 0, st>>>(x, u->cin, u->V[0], vol(u->X0, 16));
  layer_fwd(u, st, E0A, vol(u->X0, 16), vol(u->A0, 16));
  layer_fwd(u, st, E0B, vol(u->A0, 16), vol(u->C0, 48, 32));
  k_pool_fwd<<<eblocks(u->V[1] * 16), CTPB, 0, st>>>(vol(u->C0, 48, 32), 16, vol(u->P0, 16), N, d0[0], d0[1], d0[2]);
  layer_fwd(u, st, E1A, vol(u->P0, 16), vol(u->A1, 32));
  layer_fwd(u, st, E1B, vol(u->A1, 32), vol(u->C1, 96, 64));
  k_pool_fwd<<<eblocks(u->V[2] * 32), CTPB, 0, st>>>(vol(u->C1, 96, 64), 32, vol(u->P1, 32), N, d1[0], d1[1], d1[2]);
  layer_fwd(u, st, BA, vol(u->P1, 32), vol(u->A2, 64));
  layer_fwd(u, st, BB, vol(u->A2, 64), vol(u->B2, 64));
  k_up_fwd<<<eblocks(u->V[1] * 8), CTPB, 0, st>>>(vol(u->B2, 64), 64, vol(u->C1, 96, 0), N, d1[0], d1[1], d1[2]);
  layer_fwd(u, st, D1A, vol(u->C1, 96), vol(u->D1, 32));
  layer_fwd(u, st, D1B, vol(u->D1, 32), vol(u->E1, 32));
  k_up_fwd<<<eblocks(u->V[0] * 4), CTPB, 0, st>>>(vol(u->E1, 32), 32, vol(u->C0, 48, 0), N, d0[0], d0[1], d0[2]);
  layer_fwd(u, st, D0A, vol(u->C0, 48), vol(u->D0, 16));
  layer_fwd(u, st, D0B, vol(u->D0, 16), vol(u->E0, 16));
  const float *hw = u->theta + head_off();
  k_head_fwd<<<eblocks(u->V[0]), CTPB, 0, st>>>(vol(u->E0, 16), hw, hw + 16, u->V[0], y);
}

void backward(vos_unet *u, hipStream_t st, const float *target)
{
  const int N = u->N;
  const int *d0 = u->dd[0], *d1 = u->dd[1];
  const size_t V0 = u->V[0];
  k_mse<<<NB_BIAS, CTPB, 0, st>>>(u->yout, target, V0, u->dy, u->lpart);
  k_sum_double<<<1, CTPB, 0, st>>>(u->lpart, NB_BIAS, u->lsum);
  const float *hw = u->theta + head_off();
  k_head_bwd<<<NB_BIAS, CTPB, 0, st>>>(vol(u->E0, 16), hw, u->dy, V0, vol(u->gE0, 16), u->hpart);
  k_bias_grad_final<<<1, CTPB, 0, st>>>(u->hpart, 17, NB_BIAS, u->grad + head_off());
  layer_bwd(u, st, D0B, vol(u->D0, 16), vol(u->gE0, 16), vol(u->gD0, 16), vol(u->D0, 16));
  layer_bwd(u, st, D0A, vol(u->C0, 48), vol(u->gD0, 16), vol(u->gC0, 48), vol(u->C0, 48));
  k_up_bwd<<<eblocks(u->V[1] * 32), CTPB, 0, st>>>(vol(u->gC0, 48, 0), 32, vol(u->gE1, 32), N, d0[0], d0[1], d0[2]);
  layer_bwd(u, st, D1B, vol(u->D1, 32), vol(u->gE1, 32), vol(u->gD1, 32), vol(u->D1, 32));
  layer_bwd(u, st, D1A, vol(u->C1, 96), vol(u->gD1, 32), vol(u->gC1, 96), vol(u->C1, 96));
  k_up_bwd<<<eblocks(u->V[2] * 64), CTPB, 0, st>>>(vol(u->gC1, 96, 0), 64, vol(u->gB2, 64), N, d1[0], d1[1], d1[2]);
  layer_bwd(u, st, BB, vol(u->A2, 64), vol(u->gB2, 64), vol(u->gA2, 64), vol(u->A2, 64));
  layer_bwd(u, st, BA, vol(u->P1, 32), vol(u->gA2, 64), vol(u->gP1, 32), NOMASK);
  k_pool_bwd<<<eblocks(u->V[1] * 4), CTPB, 0, st>>>(vol(u->gP1, 32), 32, vol(u->gC1, 96, 64), N, d1[0], d1[1], d1[2],
                                                     1, vol(u->C1, 96, 64));
  layer_bwd(u, st, E1B, vol(u->A1, 32), vol(u->gC1, 96, 64), vol(u->gA1, 32), vol(u->A1, 32));
  layer_bwd(u, st, E1A, vol(u->P0, 16), vol(u->gA1, 32), vol(u->gP0, 16), NOMASK);
  k_pool_bwd<<<eblocks(u->V[0] * 2), CTPB, 0, st>>>(vol(u->gP0, 16), 16, vol(u->gC0, 48, 32), N, d0[0], d0[1], d0[2],
                                                     1, vol(u->C0, 48, 32));
  layer_bwd(u, st, E0B, vol(u->A0, 16), vol(u->gC0, 48, 32), vol(u->gA0, 16), vol(u->A0, 16));
  layer_bwd(u, st, E0A, vol(u->X0, 16), vol(u->gA0, 16), NOMASK, NOMASK);
}

void refresh_weights(vos_unet *u, hipStream_t st)
{
  for (int l = 0; l < NL; ++l)
    k_weights_to_bf16<<<eblocks(wsize(l)), CTPB, 0, st>>>(u->theta + layer_off(l), LAY[l].ci, LAY[l].co, u->wf[l],
                                                          u->wd[l]);
}

vos_status copy_vec(void *dst, const void *src, size_t bytes, int on_device, bool to_dev, hipStream_t st)
{
  const hipMemcpyKind k = on_device ? hipMemcpyDeviceToDevice : (to_dev ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost);
  UN_TRY(hipMemcpyAsync(dst, src, bytes, k, st));
  UN_TRY(hipStreamSynchronize(st));
  return VOS_OK;
}

}  // namespace

namespace vosint {

void unet_dims(const vos_unet *net, int *batch, int *nz, int *ny, int *nx, int *cin)
{
  *batch = net->N;
  *nz = net->D;
  *ny = net->H;
  *nx = net->W;
  *cin = net->cin;
}
float *unet_input(vos_unet *net) { return net->xin; }
float *unet_output(vos_unet *net) { return net->yout; }

vos_status unet_forward_on(vos_unet *net, hipStream_t stream)
{
  forward(net, stream, net->xin, net->yout);
  UN_TRY(hipGetLastError());
  return VOS_OK;
}

}  // namespace vosint

extern "C" {

vos_status vos_unet_param_count(size_t *n)
{
  if (!n) return fail(VOS_ERR_ARG, "NULL output");
  *n = n_params();
  return VOS_OK;
}

vos_status vos_unet_workspace_bytes(const vos_unet_shape *shape, size_t *bytes)
{
  if (vos_status st = check_shape(shape)) return st;
  if (!bytes) return fail(VOS_ERR_ARG, "NULL output");
  vos_unet u{};
  init_dims(&u, shape);
  *bytes = layout(&u, nullptr);
  return VOS_OK;
}

vos_status vos_unet_create(const vos_unet_shape *shape, void *workspace, size_t workspace_bytes, void *hip_stream,
                           vos_unet **out)
{
  if (vos_status st = check_shape(shape)) return st;
  if (!out || !workspace) return fail(VOS_ERR_ARG, "NULL workspace or output handle");
  if ((size_t)workspace % ALIGN) return fail(VOS_ERR_ARG, "workspace must be 256-byte aligned");
  vos_unet probe{};
  init_dims(&probe, shape);
  const size_t need = layout(&probe, nullptr);
  if (workspace_bytes < need) return fail(VOS_ERR_OOM, "workspace smaller than vos_unet_workspace_bytes()");
  vos_unet *u = new vos_unet(probe);
  layout(u, (char *)workspace);
  u->stream = (hipStream_t)hip_stream;
  u->t = 0;
  u->host = nullptr;
  hipError_t e = hipHostMalloc((void **)&u->host, 4 * sizeof(double), hipHostMallocDefault);
  if (e != hipSuccess) {
    delete u;
    return fail(VOS_ERR_DEVICE, std::string("hipHostMalloc: ") + hipGetErrorString(e));
  }
  hipStream_t st = u->stream;
  e = hipMemsetAsync(u->theta, 0, n_params() * sizeof(float), st);
  if (e == hipSuccess && u->train) e = hipMemsetAsync(u->grad, 0, n_params() * sizeof(float), st);
  if (e == hipSuccess) {
    refresh_weights(u, st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    (void)hipHostFree(u->host);
    delete u;
    return fail(VOS_ERR_DEVICE, std::string("U-Net initialisation: ") + hipGetErrorString(e));
  }
  *out = u;
  return VOS_OK;
}

vos_status vos_unet_destroy(vos_unet *net)
{
  if (!net) return VOS_OK;
  (void)hipStreamSynchronize(net->stream);
  if (net->host) (void)hipHostFree(net->host);
  delete net;
  return VOS_OK;
}

vos_status vos_unet_set_params(vos_unet *net, const float *theta, int on_device)
{
  if (!net || !theta) return fail(VOS_ERR_ARG, "NULL network or parameters");
  const size_t P = n_params();
  std::vector<float> h(P);
  if (on_device) {
    UN_TRY(hipMemcpyAsync(h.data(), theta, P * sizeof(float), hipMemcpyDeviceToHost, net->stream));
    UN_TRY(hipStreamSynchronize(net->stream));
  } else {
    std::memcpy(h.data(), theta, P * sizeof(float));
  }
  for (size_t i = 0; i < P; ++i)
    if (!std::isfinite(h[i])) return fail(VOS_ERR_ARG, "non-finite parameter at index " + std::to_string(i));
  hipStream_t st = net->stream;
  UN_TRY(hipMemcpyAsync(net->theta, h.data(), P * sizeof(float), hipMemcpyHostToDevice, st));
  if (net->train) {
    UN_TRY(hipMemsetAsync(net->m, 0, P * sizeof(float), st));
    UN_TRY(hipMemsetAsync(net->v, 0, P * sizeof(float), st));
  }
  net->t = 0;
  refresh_weights(net, st);
  UN_TRY(hipGetLastError());
  UN_TRY(hipStreamSynchronize(st));
  return VOS_OK;
}

vos_status vos_unet_get_params(vos_unet *net, float *theta, int on_device)
{
  if (!net || !theta) return fail(VOS_ERR_ARG, "NULL network or output");
  return copy_vec(theta, net->theta, n_params() * sizeof(float), on_device, false, net->stream);
}

// File of a network's parameters: 8 bytes "VOSUNET1", the parameter count
// (uint64, little-endian as the host writes it), then the flat FP32 vector.
vos_status vos_unet_save(vos_unet *net, const char *path)
{
  if (!net || !path) return fail(VOS_ERR_ARG, "NULL network or path");
  const size_t P = n_params();
  std::vector<float> h(P);
  if (vos_status st = copy_vec(h.data(), net->theta, P * sizeof(float), 0, false, net->stream)) return st;
  FILE *f = std::fopen(path, "wb");
  if (!f) return fail(VOS_ERR_ARG, std::string("cannot open ") + path + " for writing");
  const char magic[8] = {'V', 'O', 'S', 'U', 'N', 'E', 'T', '1'};
  const uint64_t n = P;
  bool ok = std::fwrite(magic, 1, 8, f) == 8 && std::fwrite(&n, sizeof(n), 1, f) == 1 &&
            std::fwrite(h.data(), sizeof(float), P, f) == P;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(VOS_ERR_ARG, std::string("write to ") + path + " failed");
  return VOS_OK;
}

vos_status vos_unet_load(vos_unet *net, const char *path)
{
  if (!net || !path) return fail(VOS_ERR_ARG, "NULL network or path");
  const size_t P = n_params();
  FILE *f = std::fopen(path, "rb");
  if (!f) return fail(VOS_ERR_ARG, std::string("cannot open ") + path);
  char magic[8];
  uint64_t n = 0;
  std::vector<float> h(P);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "VOSUNET1", 8) == 0 &&
            std::fread(&n, sizeof(n), 1, f) == 1 && n == P && std::fread(h.data(), sizeof(float), P, f) == P;
  char extra;
  ok = ok && std::fread(&extra, 1, 1, f) == 0;   // nothing after the parameters
  std::fclose(f);
  if (!ok) return fail(VOS_ERR_ARG, std::string(path) + " is not a parameter file of this network");
  return vos_unet_set_params(net, h.data(), 0);
}

vos_status vos_unet_get_grads(vos_unet *net, float *grad, int on_device)
{
  if (!net || !grad) return fail(VOS_ERR_ARG, "NULL network or output");
  if (!net->train) return fail(VOS_ERR_STATE, "network planned for inference only");
  return copy_vec(grad, net->grad, n_params() * sizeof(float), on_device, false, net->stream);
}

vos_status vos_unet_forward(vos_unet *net, const float *x, float *y)
{
  if (!net || !x || !y) return fail(VOS_ERR_ARG, "NULL network, input or output");
  forward(net, net->stream, x, y);
  UN_TRY(hipGetLastError());
  return VOS_OK;
}

vos_status vos_unet_loss_grad(vos_unet *net, const float *x, const float *target, double *loss)
{
  if (!net || !x || !target) return fail(VOS_ERR_ARG, "NULL network, input or target");
  if (!net->train) return fail(VOS_ERR_STATE, "network planned for inference only");
  hipStream_t st = net->stream;
  forward(net, st, x, net->yout);
  backward(net, st, target);
  UN_TRY(hipGetLastError());
  if (loss) {
    UN_TRY(hipMemcpyAsync(net->host, net->lsum, sizeof(double), hipMemcpyDeviceToHost, st));
    UN_TRY(hipStreamSynchronize(st));
    *loss = net->host[0] / (double)net->V[0];
  }
  return VOS_OK;
}

vos_status vos_unet_adam(vos_unet *net, float lr, float beta1, float beta2, float eps)
{
  if (!net) return fail(VOS_ERR_ARG, "NULL network");
  if (!net->train) return fail(VOS_ERR_STATE, "network planned for inference only");
  if (!(lr > 0.f) || !(beta1 >= 0.f && beta1 < 1.f) || !(beta2 >= 0.f && beta2 < 1.f) || !(eps > 0.f))
    return fail(VOS_ERR_ARG, "Adam needs lr > 0, 0 <= beta1, beta2 < 1, eps > 0");
  net->t += 1;
  const float c1 = (float)(1.0 - std::pow((double)beta1, net->t));
  const float c2 = (float)(1.0 - std::pow((double)beta2, net->t));
  hipStream_t st = net->stream;
  const size_t P = n_params();
  k_adam<<<eblocks(P), CTPB, 0, st>>>(net->theta, net->grad, net->m, net->v, (int)P, lr, beta1, beta2, eps, c1, c2);
  refresh_weights(net, st);
  UN_TRY(hipGetLastError());
  return VOS_OK;
}

vos_status vos_unet_train_step(vos_unet *net, const float *x, const float *target, float lr, double *loss)
{
  if (vos_status st = vos_unet_loss_grad(net, x, target, loss)) return st;
  return vos_unet_adam(net, lr, 0.9f, 0.999f, 1e-8f);
}

}  // extern "C"
