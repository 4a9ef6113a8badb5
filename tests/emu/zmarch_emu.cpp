// CPU emulation of the z-marching kernels' memory accesses (vos_march3d.h).
//
// Built with g++ -fsanitize=address against the host stand-in for the HIP
// header (tests/emu/hip/hip_runtime.h), this runs the kernels' own source
// once per (block, thread) of the launch shapes the library uses
// (zrun_len / zrun_blocks / papply_zlen from the same header), on every level
// of the hierarchies that the library builds for a grid: the pressure
// hierarchy (FP32 and FP64), the transport hierarchy (FP64) and the three
// momentum hierarchies on the face grids (FP32 and FP64), with the fused
// two-sweep legs where the library uses them.  Every array is its
// own heap allocation of exactly the size the library gives it, and the LDS
// planes are static arrays, so AddressSanitizer reports any read or write
// outside an array or an LDS plane and the program stops with a non-zero
// status.  Without such a report it prints one line per launch and "all in
// bounds".
//
//   zmarch_emu NX NY NZ [NX NY NZ ...]
#include <array>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "vos_march3d.h"

emu_dim3 threadIdx, blockIdx, blockDim, gridDim;

using namespace vos;

namespace {

long g_launches = 0;

template <typename F>
void launch(unsigned blocks, F &&kernel, unsigned tpb = TPB)
{
  gridDim.x = blocks;
  blockDim.x = tpb;
  for (unsigned b = 0; b < blocks; ++b) {
    blockIdx.x = b;
    for (unsigned t = 0; t < tpb; ++t) {
      threadIdx.x = t;
      kernel();
    }
  }
  ++g_launches;
}

// Level dimensions as the library builds them: ceil-halve every dimension
// until a level has at most cmax cells.
std::vector<std::array<int, 3>> level_chain(int nx, int ny, int nz, int cmax, int maxlev)
{
  std::vector<std::array<int, 3>> out;
  int n[3] = {nx, ny, nz};
  while ((int)out.size() < maxlev) {
    out.push_back({n[0], n[1], n[2]});
    if ((long)n[0] * n[1] * n[2] <= cmax) break;
    for (int d = 0; d < 3; ++d) n[d] = (n[d] + 1) / 2;
  }
  return out;
}

template <typename R>
struct Arrays {
  std::vector<std::vector<R>> keep;
  R *make(size_t n)
  {
    keep.emplace_back(n, (R)0);
    return keep.back().data();
  }
};

template <typename R>
void fill_dims(MgLevel<R> &L, const std::array<int, 3> &n)
{
  for (int e = 0; e < 3; ++e) L.n[e] = n[e];
  L.nc = (unsigned)n[0] * n[1] * n[2];
  for (int d = 0; d < 3; ++d) {
    for (int e = 0; e < 3; ++e) L.fd[d][e] = n[e] + (e == d);
    L.nf[d] = (unsigned)L.fd[d][0] * L.fd[d][1] * L.fd[d][2];
  }
}

template <typename R>
std::vector<MgLevel<R>> mg_levels(Arrays<R> &A, int nx, int ny, int nz)
{
  std::vector<MgLevel<R>> lv;
  for (auto &n : level_chain(nx, ny, nz, MG_COARSE_MAX, MG_MAX_LEVELS)) {
    MgLevel<R> L{};
    fill_dims(L, n);
    for (int d = 0; d < 3; ++d) L.T[d] = A.make(L.nf[d]);
    L.diag = A.make(L.nc);
    L.x = A.make(L.nc);
    L.b = A.make(L.nc);
    L.t = A.make(L.nc);
    L.dsum = lv.empty() ? 1 : 0;
    lv.push_back(L);
  }
  return lv;
}

template <typename R>
std::vector<SLevel<R>> s_levels(Arrays<R> &A, int nx, int ny, int nz)
{
  std::vector<SLevel<R>> lv;
  for (auto &n : level_chain(nx, ny, nz, SMG_COARSE_MAX, SMG_MAX_LEVELS)) {
    SLevel<R> L{};
    for (int e = 0; e < 3; ++e) L.n[e] = n[e];
    L.nc = (unsigned)n[0] * n[1] * n[2];
    L.off = A.make(6 * (size_t)L.nc);
    L.diag = A.make(L.nc);
    L.x = A.make(L.nc);
    L.b = A.make(L.nc);
    L.t = A.make(L.nc);
    L.dif = A.make(6 * (size_t)L.nc);
    lv.push_back(L);
  }
  return lv;
}

// Every marching kernel the V-cycle may launch on each level that marches
// (vcycle's zmarch test), in every variant.
template <typename Lv, typename R>
void run_levels(const char *name, std::vector<Lv> &lv)
{
  Arrays<double> D;
  const R om = (R)0.8;
  for (size_t l = 0; l + 1 < lv.size(); ++l) {
    Lv &F = lv[l];
    Lv &C = lv[l + 1];
    if (!(F.n[0] >= ZT_X / 2 && F.n[1] >= 2 && F.n[2] >= 2)) continue;
    const int zl = zrun_len(F.n);
    const unsigned nb = zrun_blocks(F.n, zl);
    double *r64 = D.make(F.nc), *dsc = D.make(F.nc), *z = D.make(F.nc), *sc = D.make(S_COUNT);
    launch(nb, [&] { k_v_pre3d<Lv, R, RHS_R>(F, r64, nullptr, 1.0, om, zl, sc); });
    launch(nb, [&] { k_v_pre3d<Lv, R, RHS_RD>(F, r64, dsc, 1.0, om, zl, sc); });
    launch(nb, [&] { k_v_pre3d<Lv, R, RHS_B>(F, r64, nullptr, 1.0, om, zl, sc); });
    launch(nb, [&] { k_v_jacobi3d<Lv, R, false>(F, F.x, F.t, om, nullptr, nullptr, zl, sc); });
    launch(nb, [&] { k_v_jacobi3d<Lv, R, true>(F, F.x, F.t, om, z, dsc, zl, sc); });
    launch(nb, [&] { k_v_restrict3d<Lv, R>(F, C, zl, sc); });
    launch(nb, [&] { k_v_post3d<Lv, R, false>(F, C, F.t, om, nullptr, nullptr, zl, sc); });
    launch(nb, [&] { k_v_post3d<Lv, R, true>(F, C, F.t, om, z, dsc, zl, sc); });
    std::printf("  %s level %zu: %d x %d x %d, z-run %d, %u blocks: 8 launches in bounds\n", name, l, F.n[0], F.n[1],
                F.n[2], zl, nb);
    if (zfused_level(F.n)) {
      constexpr int FY = zf_rows<R>;
      // one and three resident blocks per CU of 256 CUs: long and short z-runs
      for (int slots : {256, 768}) {
        const int zf = zrun_len_fused(F.n, slots, FY);
        const unsigned nf = zrun_blocks_fused(F.n, zf, FY);
        launch(nf, [&] { k_v_down3d<Lv, R, RHS_R, false>(F, C, r64, 1.0, om, zf, sc); }, ZT_X * FY);
        launch(nf, [&] { k_v_down3d<Lv, R, RHS_B, false>(F, C, r64, 1.0, om, zf, sc); }, ZT_X * FY);
        launch(nf, [&] { k_v_up3d<Lv, R, true, false>(F, C, F.t, om, z, nullptr, r64, 1.0, zf, sc); }, ZT_X * FY);
        launch(nf, [&] { k_v_up3d<Lv, R, false, false>(F, C, F.t, om, nullptr, nullptr, nullptr, 1.0, zf, sc); },
               ZT_X * FY);
        if constexpr (std::is_same<Lv, SLevel<double>>::value) {
          // the input scaled by the level's diagonal inside the legs (transport)
          launch(nf, [&] { k_v_down3d<Lv, R, RHS_RG, false>(F, C, r64, 1.0, om, zf, sc); }, ZT_X * FY);
          launch(nf, [&] { k_v_up3d<Lv, R, true, false, true>(F, C, F.t, om, z, nullptr, r64, 1.0, zf, sc); },
                 ZT_X * FY);
          if (F.off32) {   // the variants reading the FP32 off-diagonal copies
            launch(nf, [&] { k_v_down3d<Lv, R, RHS_R, true>(F, C, r64, 1.0, om, zf, sc); }, ZT_X * FY);
            launch(nf, [&] { k_v_up3d<Lv, R, true, true>(F, C, F.t, om, z, nullptr, r64, 1.0, zf, sc); }, ZT_X * FY);
            launch(nf, [&] { k_v_down3d<Lv, R, RHS_RG, true>(F, C, r64, 1.0, om, zf, sc); }, ZT_X * FY);
            launch(nf, [&] { k_v_up3d<Lv, R, true, true, true>(F, C, F.t, om, z, nullptr, r64, 1.0, zf, sc); },
                   ZT_X * FY);
          }
        }
      }
      const int zf = zrun_len_fused(F.n, 768, FY);
      const unsigned nf = zrun_blocks_fused(F.n, zf, FY);
      std::printf("  %s level %zu fused legs: z-run %d, %u blocks (and a longer run): 8 launches in bounds\n", name, l, zf, nf);
    }
  }
}

void run_papply(int nx, int ny, int nz)
{
  Dev g{};
  g.n[0] = nx;
  g.n[1] = ny;
  g.n[2] = nz;
  g.nd = 3;
  for (int d = 0; d < 3; ++d) {
    for (int e = 0; e < 3; ++e) g.fd[d][e] = g.n[e] + (e == d);
    g.nf[d] = (unsigned)g.fd[d][0] * g.fd[d][1] * g.fd[d][2];
  }
  g.nc = (unsigned)nx * ny * nz;
  if (!papply_marching(g)) {
    std::printf("  pressure operator: not marching on this grid\n");
    return;
  }
  Arrays<double> D;
  const int zl = papply_zlen(g);
  const unsigned nb = zrun_blocks(g.n, zl);
  double *T0 = D.make(g.nf[0]), *T1 = D.make(g.nf[1]), *T2 = D.make(g.nf[2]);
  double *p = D.make(g.nc), *q = D.make(g.nc), *part = D.make(MAXB), *sc = D.make(S_COUNT);
  launch(nb, [&] { k_p_apply3d(g, T0, T1, T2, p, q, part, zl, sc); });
  std::printf("  pressure operator: z-run %d, %u blocks in bounds\n", zl, nb);
}

}  // namespace

int main(int argc, char **argv)
{
  if (argc < 4 || (argc - 1) % 3) {
    std::fprintf(stderr, "usage: %s NX NY NZ [NX NY NZ ...]\n", argv[0]);
    return 2;
  }
  for (int a = 1; a + 2 < argc; a += 3) {
    const int nx = std::atoi(argv[a]), ny = std::atoi(argv[a + 1]), nz = std::atoi(argv[a + 2]);
    std::printf("grid %d x %d x %d\n", nx, ny, nz);
    run_papply(nx, ny, nz);
    {
      Arrays<float> A;
      auto lv = mg_levels(A, nx, ny, nz);
      run_levels<MgLevel<float>, float>("pressure FP32", lv);
    }
    {
      Arrays<double> A;
      auto lv = mg_levels(A, nx, ny, nz);
      run_levels<MgLevel<double>, double>("pressure FP64", lv);
    }
    {
      Arrays<double> A;
      auto lv = s_levels(A, nx, ny, nz);
      run_levels<SLevel<double>, double>("transport FP64", lv);
    }
    {
      // mixed precision: the levels that run the fused legs smooth with FP32
      // off-diagonal copies (the finest level always carries them here)
      Arrays<double> A;
      Arrays<float> A32;
      auto lv = s_levels(A, nx, ny, nz);
      for (size_t l = 0; l < lv.size(); ++l)
        if (l == 0 || zfused_level(lv[l].n)) lv[l].off32 = A32.make(6 * (size_t)lv[l].nc);
      run_levels<SLevel<double>, double>("transport FP64, FP32 off-diagonal copies", lv);
    }
    const int fn[3][3] = {{nx + 1, ny, nz}, {nx, ny + 1, nz}, {nx, ny, nz + 1}};
    for (int d = 0; d < 3; ++d) {
      char name[64];
      {
        Arrays<float> A;
        auto lv = s_levels(A, fn[d][0], fn[d][1], fn[d][2]);
        std::snprintf(name, sizeof name, "momentum %c FP32", "xyz"[d]);
        run_levels<SLevel<float>, float>(name, lv);
      }
      {
        Arrays<double> A;
        auto lv = s_levels(A, fn[d][0], fn[d][1], fn[d][2]);
        std::snprintf(name, sizeof name, "momentum %c FP64", "xyz"[d]);
        run_levels<SLevel<double>, double>(name, lv);
      }
    }
  }
  std::printf("all in bounds (%ld launches)\n", g_launches);
  return 0;
}
