// vos_batch.hip -- many independent simulations advanced concurrently
// (include/vos_batch.h).  Host orchestration only: every instance runs the
// kernels of a standalone vos_sim on its own stream; a pool of worker threads
// keeps several instances in flight so that their kernels overlap.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "vos_batch.h"
#include "vos_internal.h"

using vosint::fail;

namespace {

constexpr size_t ALIGN = 256;
constexpr int MAX_INSTANCES = 4096;
constexpr int MAX_WORKERS = 64;

size_t round_up(size_t b) { return (b + ALIGN - 1) / ALIGN * ALIGN; }

}  // namespace

struct vos_batch {
  int n = 0;
  int workers = 1;
  std::vector<vos_sim *> sims;
  std::vector<hipStream_t> streams;
  std::vector<size_t> cells;
  std::vector<int> order;       // instances by decreasing cell count
};

namespace {

void destroy_all(vos_batch *b)
{
  for (vos_sim *s : b->sims)
    if (s) vos_destroy(s);
  for (hipStream_t st : b->streams)
    if (st) (void)hipStreamDestroy(st);
  b->sims.clear();
  b->streams.clear();
}

// One pass of every instance (nsteps each) on `workers` threads.
vos_status run(vos_batch *b, const double *dt, int nsteps, int flags, int workers, vos_diag *last,
               vos_status *status)
{
  const int n = b->n;
  std::vector<vos_status> st(n, VOS_OK);
  std::vector<std::string> msg(n);
  std::atomic<int> next{0};
  auto work = [&]() {
    for (;;) {
      const int k = next.fetch_add(1);
      if (k >= n) break;
      const int i = b->order[k];
      vos_diag d{};
      st[i] = vos_step(b->sims[i], dt[i], nsteps, flags, &d);
      if (st[i] != VOS_OK) msg[i] = vos_last_error();
      if (last) last[i] = d;
    }
  };
  const int w = std::max(1, std::min(workers, n));
  std::vector<std::thread> pool;
  pool.reserve(w - 1);
  for (int t = 1; t < w; ++t) pool.emplace_back(work);
  work();
  for (auto &th : pool) th.join();
  if (status)
    for (int i = 0; i < n; ++i) status[i] = st[i];
  for (int i = 0; i < n; ++i)
    if (st[i] != VOS_OK) return fail(st[i], "instance " + std::to_string(i) + ": " + msg[i]);
  return VOS_OK;
}

// Size class of an instance for the per-class check interval: log2 of its
// cell count.
int size_class(size_t cells)
{
  int c = 0;
  while (cells > 1) { cells >>= 1; ++c; }
  return c;
}

}  // namespace

extern "C" {

vos_status vos_batch_workspace_bytes(int n, const vos_grid *grids, const vos_opts *opts, size_t *bytes)
{
  if (n < 1 || n > MAX_INSTANCES) return fail(VOS_ERR_ARG, "batch size must be in [1, 4096]");
  if (!grids || !opts || !bytes) return fail(VOS_ERR_ARG, "NULL argument");
  size_t tot = 0;
  for (int i = 0; i < n; ++i) {
    size_t b = 0;
    if (vos_status st = vos_workspace_bytes(&grids[i], &opts[i], &b))
      return fail(st, "instance " + std::to_string(i) + ": " + vos_last_error());
    tot += round_up(b);
  }
  *bytes = tot;
  return VOS_OK;
}

vos_status vos_batch_create(int n, const vos_grid *grids, const vos_params *params, const vos_opts *opts,
                            void *workspace, size_t workspace_bytes, int workers, vos_batch **out)
{
  size_t need = 0;
  if (vos_status st = vos_batch_workspace_bytes(n, grids, opts, &need)) return st;
  if (!params || !out || !workspace) return fail(VOS_ERR_ARG, "NULL argument");
  if ((size_t)workspace % ALIGN) return fail(VOS_ERR_ARG, "workspace must be 256-byte aligned");
  if (workspace_bytes < need) return fail(VOS_ERR_OOM, "workspace smaller than vos_batch_workspace_bytes()");
  if (workers < 0 || workers > MAX_WORKERS) return fail(VOS_ERR_ARG, "workers must be in [0, 64]");
  vos_batch *b = new vos_batch();
  b->n = n;
  b->workers = workers ? workers : std::min(n, 8);
  b->sims.assign(n, nullptr);
  b->streams.assign(n, nullptr);
  b->cells.resize(n);
  char *base = (char *)workspace;
  size_t off = 0;
  for (int i = 0; i < n; ++i) {
    size_t bi = 0;
    vos_workspace_bytes(&grids[i], &opts[i], &bi);
    hipError_t e = hipStreamCreateWithFlags(&b->streams[i], hipStreamNonBlocking);
    if (e != hipSuccess) {
      destroy_all(b);
      delete b;
      return fail(VOS_ERR_DEVICE, std::string("hipStreamCreateWithFlags: ") + hipGetErrorString(e));
    }
    if (vos_status st = vos_create(&grids[i], &params[i], &opts[i], base + off, bi, b->streams[i], &b->sims[i])) {
      std::string m = vos_last_error();
      destroy_all(b);
      delete b;
      return fail(st, "instance " + std::to_string(i) + ": " + m);
    }
    off += round_up(bi);
    b->cells[i] = (size_t)grids[i].nx * grids[i].ny * grids[i].nz;
  }
  b->order.resize(n);
  for (int i = 0; i < n; ++i) b->order[i] = i;
  std::stable_sort(b->order.begin(), b->order.end(), [&](int a, int c) { return b->cells[a] > b->cells[c]; });
  *out = b;
  return VOS_OK;
}

vos_status vos_batch_destroy(vos_batch *b)
{
  if (!b) return VOS_OK;
  destroy_all(b);
  delete b;
  return VOS_OK;
}

vos_status vos_batch_sim(vos_batch *b, int i, vos_sim **sim)
{
  if (!b || !sim) return fail(VOS_ERR_ARG, "NULL argument");
  if (i < 0 || i >= b->n) return fail(VOS_ERR_ARG, "instance index out of range");
  *sim = b->sims[i];
  return VOS_OK;
}

vos_status vos_batch_step(vos_batch *b, const double *dt, int nsteps, int flags, vos_diag *last, vos_status *status)
{
  if (!b || !dt) return fail(VOS_ERR_ARG, "NULL argument");
  if (nsteps < 0) return fail(VOS_ERR_ARG, "nsteps must be >= 0");
  return run(b, dt, nsteps, flags, b->workers, last, status);
}

vos_status vos_batch_tune(vos_batch *b, const double *dt, int probe_steps, int *workers, double *best_ms)
{
  if (!b || !dt) return fail(VOS_ERR_ARG, "NULL argument");
  if (probe_steps < 1 || probe_steps > 100) return fail(VOS_ERR_ARG, "probe_steps must be in [1, 100]");
  auto time_pass = [&](int w, double *ms) -> vos_status {
    const auto t0 = std::chrono::steady_clock::now();
    vos_status st = run(b, dt, probe_steps, VOS_FREEZE_SOLID, w, nullptr, nullptr);
    const auto t1 = std::chrono::steady_clock::now();
    *ms = std::chrono::duration<double, std::milli>(t1 - t0).count() / probe_steps;
    return st;
  };
  // warm-up pass: captures every instance's graphs with the current settings
  double ms = 0.0;
  if (vos_status st = time_pass(b->workers, &ms)) return st;
  // 1. worker count
  const int wmax = std::min(MAX_WORKERS, std::max(b->workers, std::min(b->n, 16)));
  int best_w = b->workers;
  double best = 0.0;
  if (vos_status st = time_pass(best_w, &best)) return st;
  for (int w = 1; w <= wmax; w *= 2) {
    if (w == best_w) continue;
    if (vos_status st = time_pass(w, &ms)) return st;
    if (ms < best) { best = ms; best_w = w; }
  }
  b->workers = best_w;
  // 2. Krylov check interval per size class
  std::vector<int> classes;
  for (int i = 0; i < b->n; ++i) classes.push_back(size_class(b->cells[i]));
  std::vector<int> uniq = classes;
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  const int cands[5] = {2, 4, 8, 16, 32};
  for (int cls : uniq) {
    int cur = 0, cc = 0;
    for (int i = 0; i < b->n; ++i)
      if (classes[i] == cls) { vosint::get_tuning(b->sims[i], &cur, &cc); break; }
    int keep = cur;
    for (int ce : cands) {
      if (ce == cur) continue;
      for (int i = 0; i < b->n; ++i)
        if (classes[i] == cls) {
          int c0, k0;
          vosint::get_tuning(b->sims[i], &c0, &k0);
          if (vos_status st = vosint::set_tuning(b->sims[i], ce, k0)) return st;
        }
      double t1 = 0.0;
      if (vos_status st = time_pass(b->workers, &t1)) return st;   // captures the new chunk length
      if (vos_status st = time_pass(b->workers, &ms)) return st;   // replays
      if (ms < best) { best = ms; keep = ce; }
    }
    for (int i = 0; i < b->n; ++i)
      if (classes[i] == cls) {
        int c0, k0;
        vosint::get_tuning(b->sims[i], &c0, &k0);
        if (c0 != keep)
          if (vos_status st = vosint::set_tuning(b->sims[i], keep, k0)) return st;
      }
  }
  // 3. tile shape of the 2-D tiled V-cycle legs per size class: the level size
  // from which they take the tall tiles (the smaller, more numerous tiles
  // suit the latency-bound middle levels of small grids)
  const unsigned tcands[4] = {1u << 16, 1u << 18, 1u << 20, 0xffffffffu};
  for (int cls : uniq) {
    unsigned keep = 0;
    for (int i = 0; i < b->n; ++i)
      if (classes[i] == cls) { keep = vosint::get_tile_big(b->sims[i]); break; }
    const unsigned cur = keep;
    for (unsigned tb : tcands) {
      if (tb == cur) continue;
      for (int i = 0; i < b->n; ++i)
        if (classes[i] == cls)
          if (vos_status st = vosint::set_tile_big(b->sims[i], tb)) return st;
      double t1 = 0.0;
      if (vos_status st = time_pass(b->workers, &t1)) return st;   // captures the new cycles
      if (vos_status st = time_pass(b->workers, &ms)) return st;   // replays
      if (ms < best) { best = ms; keep = tb; }
    }
    for (int i = 0; i < b->n; ++i)
      if (classes[i] == cls)
        if (vos_status st = vosint::set_tile_big(b->sims[i], keep)) return st;
  }
  if (workers) *workers = b->workers;
  if (best_ms) *best_ms = best;
  return VOS_OK;
}

vos_status vos_batch_tuning(vos_batch *b, int i, int *check_every, unsigned *tile_big_cells)
{
  if (!b) return fail(VOS_ERR_ARG, "NULL batch");
  if (i < 0 || i >= b->n) return fail(VOS_ERR_ARG, "instance index out of range");
  int ce = 0, cc = 0;
  vosint::get_tuning(b->sims[i], &ce, &cc);
  if (check_every) *check_every = ce;
  if (tile_big_cells) *tile_big_cells = vosint::get_tile_big(b->sims[i]);
  return VOS_OK;
}

}  // extern "C"
