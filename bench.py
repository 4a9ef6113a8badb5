"""Benchmark of the Volume-of-Solid step on one MI355X.

Workload (default, the headline): the 256^3 synthetic grain pack (dx = 4 um,
overlapping spheres of log-normal radius, median 20 voxels, sigma 0.3, seed
33, to porosity 0.23, one-voxel partial-volume ramp and 1 % interface noise,
2-voxel fluid bands at inlet and outlet), driven by a constant inlet pressure
scaled to Pe = 10 (L = sqrt(8 K / phi), U = U_D / phi, phi without the bands)
with Da = 1e-2, iVoS, dt = 1 ms, dissolving.  A step is one pass of the
whole step: coefficients, momentum predictor, pressure equation
(multigrid-preconditioned CG to a 1e-8 relative residual), correction,
transport (BiCGStab), reaction and solid update.  Inputs stay resident in HBM.

Prints ONE JSON line: cell-steps/s of the mixed-precision step (FP32
multigrid inside FP64 Krylov), beside the plain-FP64 step on the same state,
VoS-psi' on the same state, the pressure-solve bandwidth, the live roofline
of the kernel that dominates the step's kernel time, the learned warm start,
the 2-D micromodel (Infinity-Cache resident), the micromodel batch, and the
CPU oracle on a bounded crop of the same pack.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per cell of one pressure PCG iteration (each array read or
# written once per launch).  Outer FP64 flexible CG: operator p + nd face T + q
# (8 + 8 nd + 8), x/r update 56 (x, p, q, r, diagonal read; x, r written),
# z.r and z.q 24, direction 24: 136 B in 2-D, 144 B in 3-D.  One V-cycle with
# w-byte levels, per fine cell: level 0 reads the FP64 residual and writes the
# FP64 result (16 B) and each level moves, per level cell,
#   2-D (one tiled kernel per leg, any number of sweeps): down leg b, diag,
#     2 face T, x, coarse b/4 (5.25 w); up leg x, coarse x/4, b, diag, 2 T,
#     result (6.25 w); the coarser levels add 1/3;
#   3-D (z-marching kernels, one per sweep, the first two down sweeps fused):
#     first down launch b, diag, 3 face T, x (6 w); each further down sweep
#     x, b, diag, 3 T, result (7 w); restriction 6 w + coarse b w/8;
#     prolongation with the first up sweep 7 w + coarse x w/8; each further up
#     sweep 7 w: (14 nu - 1.75) w, the coarser levels adding 1/7 of that.  On
#     the finest level every launch but the first forms the diagonal from the
#     faces it has loaded: 2 nu - 1 fewer reads of w.
# Pressure sweeps per leg: the library's defaults.
P_NU = {2: 4, 3: 3}


def p_iter_bytes(nd, tag, nu=None):
    nu = P_NU[nd] if nu is None else nu
    w = 4 if tag == "mixed" else 8
    cg = 8 + 8 * nd + 8 + 56 + 24 + 24
    if nd == 2:
        return cg + 16 + 11.5 * w * 4 / 3
    assert nu >= 2, "the first two 3-D down sweeps run fused"
    per_level = (14 * nu - 1.75) * w
    return cg + 16 + per_level - (2 * nu - 1) * w + per_level / 7


# Krylov iterations per captured chunk on the micromodel: the first host check
# comes after as many chunks as the last solve of the same kind took, so short
# chunks waste at most one early-exit iteration (4.00 -> 3.96 ms/step against 4).
CHECK_EVERY = 2
# ... and on the 3-D pack, whose settled, extrapolated solves take 2-9
# iterations a step (pack headline, 20 steps: 46.3 ms/step with chunks of 8,
# 47.7 with 4, 45.6 with 2, 45.7 with 1; iterations identical)
CHECK_EVERY_3D = 2
# The solves start from an extrapolation of the last steps' solutions
# (vos_opts.extrapolate = 2: 2 x^n - x^(n-1), or 3 x^n - 3 x^(n-1) + x^(n-2) where
# that order predicted the last solution better); the start-from-x^n rate is
# reported beside it.
EXTRAPOLATE = 2
# The momentum and pressure hierarchies are rebuilt every fourth step
# (vos_opts.setup_every); a solve in between is preconditioned with an earlier
# step's hierarchy and still meets its tolerance.
SETUP_EVERY = 4
# Solid-frozen steps after the flow is rescaled to the target Pe (setup_sim).
SETUP_STEPS = 3
# Per-step pressure setup (hierarchy build, right-hand side, initial residual):
P_SETUP_BYTES = {2: 150, 3: 200}


def streaming_ceiling():
    """HBM bandwidth that plain streaming kernels (torch's own reduction and
    elementwise kernels) reach on 1 GiB FP64 arrays, beyond the Infinity
    Cache: context for the roofline fractions, which stay against the
    published 8 TB/s."""
    import torch
    n = 1 << 27
    x = torch.rand(n, dtype=torch.float64, device="cuda")
    y = torch.rand(n, dtype=torch.float64, device="cuda")
    z = torch.empty_like(x)

    def timed(f, reps=10):
        f()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            f()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    read = n * 8 / timed(lambda: x.sum()) / 1e9
    triad = 3 * n * 8 / timed(lambda: torch.add(x, y, alpha=0.5, out=z)) / 1e9
    del x, y, z
    return {"read_GBs": round(read, 1), "triad_GBs": round(triad, 1), "arrays": "1 GiB FP64",
            "kernels": "torch sum, torch add"}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def setup_sim(vos, inputs, scaling, workload, pe, da, precision, model, dt, relax_steps, extrapolate=EXTRAPOLATE):
    import torch
    es, prm = inputs.workload(workload)
    nz, ny, nx = es.shape
    params = dict(prm, model=model)
    opts = vos.Opts(precision=precision, rtol_u=1e-8, rtol_p=1e-8, rtol_c=1e-8, check_every=CHECK_EVERY,
                    extrapolate=extrapolate, setup_every=SETUP_EVERY)
    sim = vos.Sim(nx, ny, nz, prm["dx"], dict(params, kc=0.0), opts)
    sim.set_solid_fraction(es)
    d = None
    for k in range(relax_steps):
        d = sim.step(dt, 1, freeze_solid=True)
    K = d["K"]
    phi = float(sim.get("eps").mean())
    ndim = 2 if nz == 1 else 3
    u_in, kc = scaling.inlet_for(pe, da, K, phi, prm["D"], ndim)
    r = u_in / prm["u_in"]
    for name in ("ux", "uy", "uz"):
        sim.set(name, sim.get(name) * r)
    sim.set("p", (sim.get("p") - prm["p_out"]) * r + prm["p_out"])
    sim.set_params(dict(params, u_in=u_in, kc=kc))
    for _ in range(SETUP_STEPS):
        sim.step(dt, 1, freeze_solid=True)
    torch.cuda.synchronize()
    return sim, es, dict(params, u_in=u_in, kc=kc), dict(K=K, phi=phi, u_in=u_in, kc=kc, ndim=ndim)


# Kernel families timed live on the pack (the pressure operator and the z-marching
# kernels of the pressure hierarchy's finest level).
PACK_TIMERS = ("c_down3d", "c_up3d", "c_pre3d", "c_sweep3d", "c_restrict3d", "c_post3d", "adr_apply",
               "p_apply", "p_pre3d", "p_sweep3d", "p_restrict3d", "p_post3d", "m_down3d", "m_up3d")
# The live roofline's kernel: the one with the most kernel time in the headline's
# timed steps on the committed trace (the fused up leg of the transport
# hierarchy's finest level, k_v_up3d<SLevel<double>>, reading the FP32 copies of
# the off-diagonals in mixed precision).
ROOFLINE_FAMILY = "c_up3d"
KERNEL_NAMES = {
    "c_down3d": "k_v_down3d<SLevel<double>> transport hierarchy, finest level (fused: two sweeps from the residual "
                "and the restriction)",
    "c_up3d": "k_v_up3d<SLevel<double>> transport hierarchy, finest level (fused: prolongation and two sweeps)",
    "m_down3d": "k_v_down3d<SLevel> x-momentum hierarchy, finest level (fused down leg)",
    "m_up3d": "k_v_up3d<SLevel> x-momentum hierarchy, finest level (fused up leg)",
    "c_pre3d": "k_v_pre3d<SLevel<double>> transport hierarchy, finest level (two sweeps from the residual)",
    "c_sweep3d": "k_v_jacobi3d<SLevel<double>> transport hierarchy, finest level (one sweep)",
    "c_restrict3d": "k_v_restrict3d<SLevel<double>> transport hierarchy, finest level (residual restriction)",
    "c_post3d": "k_v_post3d<SLevel<double>> transport hierarchy, finest level (prolongation + first up sweep)",
    "adr_apply": "k_adr_apply transport operator (FP64)",
    "p_apply": "k_p_apply3d pressure operator (FP64)",
    "p_pre3d": "k_v_pre3d<MgLevel> pressure hierarchy, finest level",
    "p_sweep3d": "k_v_jacobi3d<MgLevel> pressure hierarchy, finest level",
    "p_restrict3d": "k_v_restrict3d<MgLevel> pressure hierarchy, finest level",
    "p_post3d": "k_v_post3d<MgLevel> pressure hierarchy, finest level",
}
# Settling of the pack's flow before it is rescaled to the target Pe: frozen-solid
# iterations (vos_initialize) at a short step until the face velocities change
# by at most PACK_SETTLE_TOL relative per iteration.  Each step of the
# projection is one SIMPLE-like iteration whose implicit relaxation is set by
# rho / dt against the viscous coupling mu / dx^2 (60x larger at dt = 1 ms,
# dx = 4 um): at 1 ms the permeability approaches its steady value by ~1.5 %
# per step, at 60 us it halves its distance every ~9 steps.
PACK_SETTLE_DT = 6e-5
PACK_SETTLE_TOL = 1e-4
PACK_SETTLE_MAX = 150


def setup_pack(vos, inputs, scaling, n, pe, da, precision, model, dt, extrapolate=EXTRAPOLATE):
    """The grain pack under a constant inlet pressure: settle the flow to its
    steady state with the solid frozen and no reaction, measure K and phi (phi without the 2-voxel
    inlet/outlet bands), then rescale the (Stokes-linear) flow to the pressure
    drop that gives Pe and set k_c for Da."""
    import torch
    es = inputs.sphere_pack(n, seed=33)
    prm = dict(inputs.BASE_PARAMS, dx=4e-6)
    p0 = 1.0
    params = dict(prm, model=model, drive=1, p_in=prm["p_out"] + p0)
    opts = vos.Opts(precision=precision, rtol_u=1e-8, rtol_p=1e-8, rtol_c=1e-8, maxit_p=6000,
                    check_every=CHECK_EVERY_3D, extrapolate=extrapolate, setup_every=SETUP_EVERY)
    sim = vos.Sim(n, n, n, prm["dx"], dict(params, kc=0.0), opts)
    sim.set_solid_fraction(es)
    t0 = time.perf_counter()
    dinit = sim.initialize(PACK_SETTLE_DT, PACK_SETTLE_MAX, PACK_SETTLE_TOL)
    d = sim.step(PACK_SETTLE_DT, 1, freeze_solid=True)
    settle = dict(iterations=dinit["outer_its"] + 1, last_rel_change=dinit["outer_res"],
                  seconds=round(time.perf_counter() - t0, 1))
    K = d["K"]
    phi = float(sim.get("eps")[:, :, 2:-2].mean())
    dp, kc = scaling.pressure_drop_for(pe, da, K, phi, prm["D"], prm["mu"], n * prm["dx"], 3)
    r = dp / p0
    for name in ("ux", "uy", "uz"):
        sim.set(name, sim.get(name) * r)
    sim.set("p", (sim.get("p") - prm["p_out"]) * r + prm["p_out"])
    params = dict(params, p_in=prm["p_out"] + dp, kc=kc)
    sim.set_params(params)
    for _ in range(SETUP_STEPS):
        sim.step(dt, 1, freeze_solid=True)
    torch.cuda.synchronize()
    return sim, es, params, dict(K=K, phi=phi, dp=dp, kc=kc, ndim=3, settle=settle)


# Host clocks at the synchronised start and end of each timed run, by leg name
# (bench.py --trace-window writes them for trace_window.py to cut a kernel trace).
TRACE_WINDOWS = {}


def _clocks():
    return time.clock_gettime_ns(time.CLOCK_MONOTONIC), time.clock_gettime_ns(time.CLOCK_BOOTTIME)


def timed_steps(sim, dt, steps, warmup, leg=None):
    import torch
    for _ in range(warmup):
        sim.step(dt)
    diags = []
    torch.cuda.synchronize()
    c0 = _clocks()
    t0 = time.perf_counter()
    for _ in range(steps):
        diags.append(sim.step(dt))
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    c1 = _clocks()
    if leg:
        TRACE_WINDOWS[leg] = {"monotonic": [c0[0], c1[0]], "boottime": [c0[1], c1[1]], "steps": steps}
    return el, diags


def measured_traffic(family):
    """HBM bytes per launch from the committed rocprofv3 FETCH_SIZE/WRITE_SIZE
    runs (profiles/hbm_traffic.json), or None if the kernels changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except OSError:
        return None
    from paper_2204_07019_amd.trace_window import kernel_sources_sha
    if t.get("csrc_sha") != kernel_sources_sha():
        return None
    k = t.get("kernels", {}).get(family)
    return round(k["traffic_bytes"]) if k and "traffic_bytes" in k else None


def roofline(sim, family, reps=200, with_traffic=True):
    """Live roofline of one kernel family: back-to-back launches on the
    state the timed steps left, between two HIP events on the sim's stream."""
    t = sim.time_kernel(family, reps)
    achieved = t["bytes"] / (t["avg_ms"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4),
            "traffic": measured_traffic(family) if with_traffic else None, "kernel": family,
            "kernel_name": KERNEL_NAMES.get(family, family),
            "avg_launch_us": round(t["avg_ms"] * 1e3, 3), "bytes_per_launch": round(t["bytes"])}


BATCH_SIZES = ((256, 128), (512, 256), (768, 384), (1024, 512))


def batch_bench(vos, inputs, scaling, n, steps, dt, seed=2, relax=5):
    """Many micromodels at once: n RSA-disc micromodels with sizes drawn from
    BATCH_SIZES, Pe ~ logU[0.1, 100], Da ~ logU[1e-3, 1], iVoS, mixed
    precision, advanced together by the batch API after autotuning."""
    import numpy as np
    import torch
    from paper_2204_07019_amd.batch import Batch
    rng = np.random.default_rng(seed)
    picks = rng.integers(0, len(BATCH_SIZES), n)
    pe = 10 ** rng.uniform(-1, 2, n)
    da = 10 ** rng.uniform(-3, 0, n)
    base = dict(inputs.BASE_PARAMS, model=0)
    specs = [(BATCH_SIZES[k][0], BATCH_SIZES[k][1], 1, 5e-6, dict(base, kc=0.0)) for k in picks]
    opts = vos.Opts(precision=vos.MIXED, rtol_u=1e-8, rtol_p=1e-8, rtol_c=1e-8, check_every=8,
                    extrapolate=EXTRAPOLATE, setup_every=SETUP_EVERY)
    b = Batch(specs, opts)
    for i, (nx, ny, *_rest) in enumerate(specs):
        b.sims[i].set_solid_fraction(inputs.rsa_discs(nx, ny, seed=100 + i))
    d = b.step(dt, relax, freeze_solid=True)
    for i, s in enumerate(b.sims):
        phi = float(s.get("eps").mean())
        u_in, kc = scaling.inlet_for(pe[i], da[i], d[i]["K"], phi, base["D"], 2)
        r = u_in / base["u_in"]
        for f in ("ux", "uy"):
            s.set(f, s.get(f) * r)
        s.set("p", (s.get("p") - base["p_out"]) * r + base["p_out"])
        s.set_params(dict(base, u_in=u_in, kc=kc))
    b.step(dt, 2, freeze_solid=True)
    tuned = b.tune(dt, probe_steps=1)
    # the settings the tuner chose per grid size (check interval, tall-tile threshold)
    tuned["per_size"] = {}
    for i, (nx, ny, *_r) in enumerate(specs):
        tuned["per_size"].setdefault(f"{nx}x{ny}", b.tuning(i))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    diags = b.step(dt, steps)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    # the same instances advanced one after another (one host thread, no overlap
    # between instances) for the same number of steps, continuing from there
    t0 = time.perf_counter()
    for s in b.sims:
        s.step(dt, steps)
    torch.cuda.synchronize()
    el_seq = time.perf_counter() - t0
    cells = sum(nx * ny for (nx, ny, *_r) in specs)
    out = {"workload": f"{n} RSA micromodels, sizes from {['%dx%d' % s for s in BATCH_SIZES]}, "
                       f"Pe logU[0.1,100], Da logU[1e-3,1], iVoS, mixed, dt={dt:g}s, rtol 1e-8",
           "instances": n, "cells": cells, "steps": steps,
           "value": cells * steps / el, "unit": "cell-steps/s", "ms_per_batch_step": el / steps * 1e3,
           "sequential_value": cells * steps / el_seq,
           "tuned": tuned,
           "max_its_p": max(dg["it_p"] for dg in diags), "max_its_c": max(dg["it_c"] for dg in diags)}
    b.close()
    return out


# U-Net layer shapes (input, output channels) and levels, for the FLOP count.
UNET_LAYERS = ((16, 16, 0), (16, 16, 0), (16, 32, 1), (32, 32, 1), (32, 64, 2), (64, 64, 2),
               (96, 32, 1), (32, 32, 1), (48, 16, 0), (16, 16, 0))
BF16_PEAK_TFLOPS = 2500.0


def unet_flops(voxels, train):
    """Convolution FLOPs (2 per multiply-add) of one forward pass, or of one
    training step (forward + data gradient of every layer but the first +
    weight gradient)."""
    fwd = sum(2 * 27 * ci * co * voxels / 8 ** lv for ci, co, lv in UNET_LAYERS)
    if not train:
        return fwd
    dg = sum(2 * 27 * ci * co * voxels / 8 ** lv for ci, co, lv in UNET_LAYERS[1:])
    return 2 * fwd + dg


def unet_bench(inputs, n, batch_train, reps=5):
    """Forward (batch 1) and training step (batch_train) of the warm-start
    U-Net on n^3 voxels, timed with HIP events on the network's stream."""
    import ctypes as C
    import torch
    from paper_2204_07019_amd import unet as U
    out = {}
    for name, b, train in (("forward", 1, False), ("train_step", batch_train, True)):
        net = U.UNet(b, n, n, n, cin=4, train=train)
        net.set_params(inputs.unet_init(0))
        x = torch.randn(b, n, n, n, 4, device="cuda")
        t = torch.randn(b, n, n, n, device="cuda")
        y = torch.empty(b, n, n, n, device="cuda")
        torch.cuda.synchronize()
        L = U.lib()

        def run():
            if train:
                vos_rc = L.vos_unet_train_step(net._h, C.c_void_p(x.data_ptr()), C.c_void_p(t.data_ptr()),
                                               C.c_float(1e-5), None)
            else:
                vos_rc = L.vos_unet_forward(net._h, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()))
            assert vos_rc == 0, L.vos_last_error()
        run()
        net.stream.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(net.stream)
        for _ in range(reps):
            run()
        e1.record(net.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / reps
        tf = unet_flops(b * n ** 3, train) / ms / 1e9
        out[name] = {"batch": b, "voxels": b * n ** 3, "ms": round(ms, 3), "TFLOPs": round(tf, 1),
                     "frac_bf16_peak": round(tf / BF16_PEAK_TFLOPS, 4)}
        net.close()
    return out


def learned_3d(vos, inputs, n, dt, snapshots=60, iters=400, steps=10):
    """Learned warm start beside plain FP64 and mixed precision on an n^3 grain
    pack (median radius n/10, porosity 0.3, seed 34, dx = 4 um, iVoS): the
    network is trained by the library's own kernels on snapshots the solver
    produced, then three copies of the same state take `steps` steps each at
    an equal 1e-8 pressure residual."""
    import torch
    from paper_2204_07019_amd import unet as U
    from paper_2204_07019_amd import warmstart as W
    es = inputs.sphere_pack(n, seed=34, median_r=n / 10.0, porosity=0.3)
    prm = dict(inputs.BASE_PARAMS, dx=4e-6, model=0)

    def make(prec, extrapolate=0):
        return vos.Sim(n, n, n, prm["dx"], prm, vos.Opts(precision=prec, rtol_u=1e-8, rtol_p=1e-8, rtol_c=1e-8,
                                                          maxit_p=6000, extrapolate=extrapolate))
    base = make(vos.MIXED)
    base.set_solid_fraction(es)
    base.step(dt, 3, freeze_solid=True)
    t0 = time.perf_counter()
    data = W.collect(base, snapshots, dt, U.UNet(1, n, n, n, cin=4, train=False))
    t_collect = time.perf_counter() - t0
    net = U.UNet(2, n, n, n, cin=4, train=True)
    net.set_params(inputs.unet_init(1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = W.train(net, data, iters, lr=1e-3, log_every=iters // 4)
    t_train = time.perf_counter() - t0
    state = {k: base.get(k) for k in ("eps", "ux", "uy", "uz", "p", "c")}
    base.close()
    inf = U.UNet(1, n, n, n, cin=4, train=False)
    inf.set_params(net.get_params())
    net.close()
    out = {"workload": f"pack {n}^3 median radius {n / 10:g} porosity 0.3 seed 34, iVoS, dt={dt:g}s, rtol 1e-8",
           "snapshots": snapshots, "train_iters": iters, "train_loss": [round(l, 4) for _, l in hist],
           "collect_s": round(t_collect, 2), "train_s": round(t_train, 2)}
    for name, prec, learned, ex in (("plain_fp64", vos.FP64, False, 0), ("mixed", vos.MIXED, False, 0),
                                    ("mixed_learned", vos.MIXED, True, 0),
                                    ("mixed_extrapolated", vos.MIXED, False, EXTRAPOLATE)):
        s = make(prec, ex)
        for k, v in state.items():
            s.set(k, v)
        if learned:
            U.attach(s, inf, gain=data.gain, use_guess=True)
        s.step(dt)   # warm-up (graph capture; the extrapolation's first history point)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ds = [s.step(dt) for _ in range(steps)]
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        out[name] = {"cell_steps_per_s": n ** 3 * steps / el, "ms_per_step": el / steps * 1e3,
                     "pressure_its_per_step": sum(d["it_p"] for d in ds) / steps,
                     "pressure_ms_per_step": sum(d["t_ms"][2] for d in ds) / steps}
        if learned:
            out[name]["guess_accepted"] = sum(1 for d in ds if d["guess"] == 1)
            out[name]["error_drop_mean"] = sum(d["guess_error_drop"] for d in ds) / steps
        s.close()
    inf.close()
    return out


def _oracle_pack_crop(job):
    """One oracle run (plain C, one thread) on an n_crop^3 corner of the 256^3
    pack: a cold-start step, then steps until budget_s of stepping."""
    n_crop, params, dt, budget_s = job
    import oracle
    from paper_2204_07019_amd import inputs
    es = np.ascontiguousarray(inputs.sphere_pack(256, seed=33)[:n_crop, :n_crop, :n_crop])
    keys = ("mu", "rho", "D", "k0", "kc", "Vm", "zeta", "c_in", "eps_min", "u_in", "p_out", "model", "drive")
    kw = {k: params[k] for k in keys}
    kw["p_in"] = params["p_out"] + (params["p_in"] - params["p_out"]) * n_crop / 256.0
    prob = oracle.Problem(nx=n_crop, ny=n_crop, nz=n_crop, dx=params["dx"], **kw, rtol_u=1e-8, rtol_p=1e-8,
                          rtol_c=1e-8)
    st = oracle.initial_state(prob, es)
    t0 = time.perf_counter()
    oracle.step(prob, st, dt, check=False)           # leave the cold start
    t_cold = time.perf_counter() - t0
    nsteps, t = 0, 0.0
    while t < budget_s and nsteps < 20:
        t0 = time.perf_counter()
        oracle.step(prob, st, dt, check=False)
        t += time.perf_counter() - t0
        nsteps += 1
    return n_crop ** 3 * nsteps, t, nsteps, t_cold


def cpu_baseline_pack(n_crop, params, dt, budget_s):
    """The oracle on a bounded sample of the headline workload: an n_crop^3
    corner of the 256^3 pack with the same parameters (the inlet pressure drop
    scaled with the crop's length, so the same pressure gradient), from rest.
    Once on one thread, then as many independent copies as the host offers
    cores (at most 16), side by side: the whole host's oracle throughput."""
    import multiprocessing as mp
    import oracle
    oracle.build(force=False)
    cs, t, nsteps, t_cold = _oracle_pack_crop((n_crop, params, dt, budget_s / 2))
    one = cs / t
    procs = max(1, min(16, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()))
    with mp.get_context("spawn").Pool(procs) as pool:
        t0 = time.perf_counter()
        res = pool.map(_oracle_pack_crop, [(n_crop, params, dt, budget_s / 2)] * procs)
        wall = time.perf_counter() - t0
    # each copy's stepping rate, summed (their cold steps excluded as in the single run)
    allc = sum(r[0] / r[1] for r in res)
    return {"value": allc, "unit": "cell-steps/s", "cores": procs, "kind": "oracle",
            "single_thread": {"value": one, "cores": 1},
            "sample": f"{nsteps} steps of a {n_crop}^3 corner of the 256^3 pack (same parameters, pressure drop "
                      f"scaled to the crop length, FP64 plain C one thread per copy, rtol 1e-8, Jacobi-PCG / "
                      f"BiCGStab) after a {t_cold:.1f} s cold-start step; the flow starts from rest, where the "
                      f"GPU's is settled; value: {procs} copies side by side ({wall:.0f} s wall)"}


def cpu_baseline(workload, params, dt, budget_s):
    """The oracle (plain C, one thread) on a bounded sample of a 2-D
    workload: a crop of the same geometry, one step at a time until the
    budget is used."""
    import oracle
    from paper_2204_07019_amd import inputs
    oracle.build(force=False)
    es, prm = inputs.workload(workload)
    nz, ny, nx = es.shape
    cy, cx = max(1, ny // 4), max(2, nx // 4)
    crop = np.ascontiguousarray(es[:, :cy, :cx])
    keys = ("mu", "rho", "D", "k0", "kc", "Vm", "zeta", "c_in", "eps_min", "u_in", "p_out", "model")
    prob = oracle.Problem(nx=crop.shape[2], ny=crop.shape[1], nz=1, dx=prm["dx"],
                          **{k: params[k] for k in keys}, rtol_u=1e-8, rtol_p=1e-8, rtol_c=1e-8)
    st = oracle.initial_state(prob, crop)
    oracle.step(prob, st, dt, check=False)           # leave the cold start
    n, t = 0, 0.0
    while t < budget_s and n < 50:
        t0 = time.perf_counter()
        oracle.step(prob, st, dt, check=False)
        t += time.perf_counter() - t0
        n += 1
    cells = prob.nx * prob.ny * prob.nz
    return {"value": cells * n / t, "unit": "cell-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} steps of a {prob.nx}x{prob.ny} crop of the {workload} geometry "
                      f"(same parameters, FP64, single-threaded C), {t:.1f} s"}


FIELDS = ("eps", "ux", "uy", "uz", "p", "c")


def run_summary(diags, el, cells, steps, nd, tag, info=None, params=None):
    """Rates, iterations and the pressure stage's algorithmic bandwidth of a timed run."""
    its_p = sum(d["it_p"] for d in diags)
    its64 = sum(d["it_p"] if tag == "fp64" else d["it_p_fp64"] for d in diags)
    t_p = sum(d["t_ms"][2] for d in diags) * 1e-3
    pb = cells * (p_iter_bytes(nd, tag) * (its_p - its64) + p_iter_bytes(nd, "fp64") * its64 +
                  P_SETUP_BYTES[nd] * len(diags))
    out = {"value": cells * steps / el, "ms_per_step": el / steps * 1e3,
           "pressure_its_per_step": its_p / len(diags), "pressure_its_fp64_hierarchy": its64 / len(diags),
           "momentum_its_per_step": [sum(d["it_u"][k] for d in diags) / len(diags) for k in range(3)],
           "transport_its_per_step": sum(d["it_c"] for d in diags) / len(diags),
           "pressure_ms_per_step": t_p / len(diags) * 1e3,
           "pressure_GBs_algorithmic": round(pb / t_p / 1e9, 1) if t_p > 0 else None,
           "pressure_frac_hbm": round(pb / t_p / 1e9 / HBM_PEAK_GBS, 4) if t_p > 0 else None,
           "stage_ms": [round(sum(d["t_ms"][k] for d in diags) / len(diags), 3) for k in range(6)],
           # worst per-step closure of the acid and solid balances (relative), a
           # check of the timed steps themselves at the run's size
           "max_balance_rel": {"acid": max(abs(d["acid_balance_rel"]) for d in diags),
                               "solid": max(abs(d["solid_balance_rel"]) for d in diags)}}
    if info is not None and params is not None:
        from paper_2204_07019_amd import scaling
        last = diags[-1]
        sc = scaling.scales(last["K"], info["phi"], last["U_D"], params["D"], params["kc"], nd)
        out["achieved"] = {"Pe": round(sc["Pe"], 3), "Da": round(sc["Da"], 5), "U_D": last["U_D"], "K": last["K"],
                           "solid_rate_mol_s": last["solid_rate"], "max_deps": last["max_deps"]}
    return out


def pack_leg(vos, inputs, scaling, args):
    """The headline (mixed precision, iVoS) on the pack, its live roofline,
    then the plain-FP64 step and VoS-psi' continuing from the same relaxed
    state for the same number of steps."""
    import torch
    n = args.n3d
    cells = n ** 3
    log(f"pack {n}^3: setup (frozen flow, Pe={args.pe:g}, Da={args.da:g})")
    sim, es, params, info = setup_pack(vos, inputs, scaling, n, args.pe, args.da, vos.MIXED, args.model, args.dt)
    log(f"K={info['K']:.3e} phi={info['phi']:.3f} dp={info['dp']:.3e} Pa kc={info['kc']:.3e}")
    state = {k: sim.get(k) for k in FIELDS}
    el, diags = timed_steps(sim, args.dt, args.steps, args.warmup, leg="headline")
    head = run_summary(diags, el, cells, args.steps, 3, "mixed", info, params)
    log(f"mixed iVoS: {head['ms_per_step']:.1f} ms/step, {head['value']:.3e} cell-steps/s, "
        f"{head['pressure_its_per_step']:.1f} pressure its/step")
    roof = roofline(sim, args.timer)
    others = {k: roofline(sim, k, reps=20) for k in PACK_TIMERS if k != args.timer}
    sim.close()
    del sim
    torch.cuda.empty_cache()
    comps = {}
    for name, prec, model in (("plain_fp64", vos.FP64, args.model), ("psi_prime_mixed", vos.MIXED, 2)):
        if args.skip_plain or args.only_headline:
            break
        opts = vos.Opts(precision=prec, rtol_u=1e-8, rtol_p=1e-8, rtol_c=1e-8, maxit_p=6000,
                        check_every=CHECK_EVERY_3D, extrapolate=EXTRAPOLATE, setup_every=SETUP_EVERY)
        s2 = vos.Sim(n, n, n, params["dx"], dict(params, model=model), opts)
        for k, v in state.items():
            s2.set(k, v)
        el2, d2 = timed_steps(s2, args.dt, args.steps, args.warmup, leg=name)
        comps[name] = run_summary(d2, el2, cells, args.steps, 3, "fp64" if prec == vos.FP64 else "mixed",
                                  info, dict(params, model=model))
        log(f"{name}: {comps[name]['ms_per_step']:.1f} ms/step, {comps[name]['value']:.3e} cell-steps/s")
        s2.close()
        del s2
        torch.cuda.empty_cache()
    return head, roof, others, comps, params, info, cells


def micromodel_sweep(vos, inputs, scaling, steps, dt):
    """The 1024x512 micromodel configuration's runs: Pe in {0.1, 10, 100} x Da
    in {1e-3, 1e-1}, plain FP64 and mixed precision, `steps` dissolving steps
    each (after 3 untimed ones).  Cache-resident rates (~100 MB of state)."""
    import torch
    runs = []
    for pe in (0.1, 10.0, 100.0):
        for da in (1e-3, 1e-1):
            for prec, tag in ((vos.FP64, "fp64"), (vos.MIXED, "mixed")):
                sim, es, params, info = setup_sim(vos, inputs, scaling, "micromodel", pe, da, prec, 0, dt, 40)
                nz, ny, nx = es.shape
                el, diags = timed_steps(sim, dt, steps, 3)
                r = run_summary(diags, el, nx * ny * nz, steps, 2, tag, info, params)
                runs.append({"Pe": pe, "Da": da, "precision": tag, "value": r["value"],
                             "ms_per_step": round(r["ms_per_step"], 4),
                             "pressure_its_per_step": r["pressure_its_per_step"],
                             "momentum_its_per_step": r["momentum_its_per_step"][:2],
                             "transport_its_per_step": r["transport_its_per_step"],
                             "achieved": {k: r["achieved"][k] for k in ("Pe", "Da")},
                             "porosity_change": float(sim.get("eps").mean()) - info["phi"]})
                sim.close()
                del sim
                torch.cuda.empty_cache()
    return {"workload": f"micromodel 1024x512 dx=5um RSA discs seed 11, iVoS, dt={dt:g}s, rtol 1e-8, "
                        f"{steps} dissolving steps per run; Infinity-Cache (MALL) resident",
            "steps": steps, "runs": runs}


def micromodel_leg(vos, inputs, scaling, steps, warmup, dt):
    """The 1024x512 micromodel (Pe = 10, Da = 0.1), mixed precision: its
    ~100 MB state lives in the 256 MB Infinity Cache, so its rates are
    cache-resident, not HBM figures."""
    sim, es, params, info = setup_sim(vos, inputs, scaling, "micromodel", 10.0, 0.1, vos.MIXED, 0, dt, 40)
    nz, ny, nx = es.shape
    el, diags = timed_steps(sim, dt, steps, warmup)
    out = run_summary(diags, el, nx * ny * nz, steps, 2, "mixed")
    out["workload"] = (f"micromodel {nx}x{ny} dx=5um RSA discs seed 11, iVoS, Pe=10 Da=0.1, dt={dt:g}s, "
                       "rtol 1e-8, mixed precision; Infinity-Cache (MALL) resident")
    out["roofline_mall_resident"] = {k: roofline(sim, k, with_traffic=False) for k in ("v_down", "v_up")}
    for v in out["roofline_mall_resident"].values():
        v["bound"] = "mall"
    sim.close()
    return out


# Upscaling workload: quasi-static steps (the SIMPLE loop of Appendix B to an
# initial relative residual of UPSCALING_OUTER_TOL per solve, relaxation 0.7 /
# 0.3), the solid step set by Appendix D's bound on the change of the fluid
# fraction (the nominal step UPSCALING_DT only caps it).
UPSCALING_DEPS_MAX = 0.005
UPSCALING_DT = 1e3
UPSCALING_OUTER_TOL = 1e-6


def upscaling_leg(vos, inputs, scaling, budget_s, target_rel, dt_setup):
    """A long dissolution run of the 1024x512 micromodel (iVoS, Pe 10, Da 0.1,
    mixed precision) until its porosity has grown by target_rel (or the wall
    time budget ends), with the K(phi) and alpha(phi) power-law fits."""
    from paper_2204_07019_amd import upscaling as U
    import torch
    sim, es, params, info = setup_sim(vos, inputs, scaling, "micromodel", 10.0, 0.1, vos.MIXED, 0, dt_setup, 40)
    nz, ny, nx = es.shape
    state = {k: sim.get(k) for k in ("eps", "ux", "uy", "p", "c")}
    dx = sim.grid.dx
    sim.close()
    del sim
    opts = vos.Opts(precision=vos.MIXED, rtol_u=1e-8, rtol_p=1e-8, rtol_c=1e-8, check_every=CHECK_EVERY,
                    extrapolate=0, setup_every=SETUP_EVERY, deps_max=UPSCALING_DEPS_MAX, simple=1,
                    outer_max=300, outer_tol=UPSCALING_OUTER_TOL, relax_u=0.7, relax_p=0.3, relax_c=1.0)
    s = vos.Sim(nx, ny, nz, dx, params, opts)
    for k, v in state.items():
        s.set(k, v)
    phi0 = float(state["eps"].mean().item())
    rec = U.run(s, UPSCALING_DT, 1000000, target_porosity=phi0 * (1.0 + target_rel), time_budget=budget_s)
    s.close()
    torch.cuda.empty_cache()
    n = len(rec["phi"])
    out = {"workload": f"micromodel {nx}x{ny} dx=5um RSA discs seed 11, iVoS, Pe=10 Da=0.1, mixed precision, "
                       f"quasi-static SIMPLE steps (relaxation 0.7/0.3, outer tolerance {UPSCALING_OUTER_TOL:g}), "
                       f"deps_max={UPSCALING_DEPS_MAX}",
           "steps": n, "wall_s": round(rec["wall_s"], 2), "ms_per_step": round(rec["wall_s"] / max(n, 1) * 1e3, 3),
           "cell_steps_per_s": nx * ny * n / rec["wall_s"], "phi_start": phi0, "phi_end": rec["phi_end"],
           "target_phi": phi0 * (1.0 + target_rel), "reached": rec["phi_end"] >= phi0 * (1.0 + target_rel),
           "simulated_s": float(rec["t"][-1]) if n else 0.0,
           "outer_its_per_step": float(np.mean(rec["outer_its"])) if n else 0.0}
    if n >= 6:
        for y in ("K", "alpha"):
            c, e, rms = U.fit_power_law(rec["phi"], rec[y])
            out[f"{y}_fit"] = {"C": c, "exponent": e, "rms_log": rms}
            k, f1, f2 = U.fit_two_power_laws(rec["phi"], rec[y], min_points=max(3, n // 10))
            out[f"{y}_two_laws"] = {"split_phi": float(rec["phi"][k]), "first": {"C": f1[0], "exponent": f1[1]},
                                    "second": {"C": f2[0], "exponent": f2[1]}}
        sel = np.linspace(0, n - 1, min(n, 12)).astype(int)
        out["samples"] = {k: [float(rec[k][i]) for i in sel] for k in ("phi", "K", "alpha")}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)   # the pack configuration's 100 steps
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--pe", type=float, default=10.0)
    ap.add_argument("--da", type=float, default=1e-2)
    ap.add_argument("--model", type=int, default=0)
    ap.add_argument("--dt", type=float, default=1e-3)
    ap.add_argument("--n3d", type=int, default=256)
    ap.add_argument("--timer", default=ROOFLINE_FAMILY, help="kernel family of the live roofline")
    ap.add_argument("--only-headline", action="store_true",
                    help="the headline pack run alone (profiling): no comparisons or secondary legs")
    ap.add_argument("--skip-plain", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--cpu-crop", type=int, default=40)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-micromodel", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the many-micromodel batch")
    ap.add_argument("--no-micromodel-sweep", action="store_true",
                    help="skip the micromodel runs over Pe, Da and precision")
    ap.add_argument("--batch-n", type=int, default=64)
    ap.add_argument("--batch-steps", type=int, default=100)
    ap.add_argument("--no-unet", action="store_true", help="skip the U-Net timing")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm start comparison")
    ap.add_argument("--no-upscaling", action="store_true", help="skip the long upscaling run")
    ap.add_argument("--upscaling-budget", type=float, default=40.0, help="wall seconds of the upscaling run")
    ap.add_argument("--only-upscaling", action="store_true", help="the upscaling run alone")
    ap.add_argument("--n-learned", type=int, default=128)
    ap.add_argument("--unet-n", type=int, default=128)
    ap.add_argument("--trace-window", default=None,
                    help="write the host-clock windows of the timed runs to this JSON file")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only copy 1 GiB device-to-device 5 times (HBM counter calibration)")
    args = ap.parse_args()

    if args.calibrate_copy:
        import torch
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_per_launch": src.numel() * 8, "launches": 5}))
        return

    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the multi-GPU path "
              "(slabs along the flow with halo exchange) is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2204_07019_amd import inputs, scaling, vos
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    vos.lib()

    if args.only_upscaling:
        print(json.dumps({"upscaling": upscaling_leg(vos, inputs, scaling, args.upscaling_budget, 0.2, args.dt)}))
        return
    head, roof, others, comps, params, info, cells = pack_leg(vos, inputs, scaling, args)
    n = args.n3d
    extra = {}
    if not args.only_headline:
        if not args.no_learned:
            log(f"learned warm start {args.n_learned}^3")
            extra["learned_3d"] = learned_3d(vos, inputs, args.n_learned, 2e-3)
            log("learned: " + ", ".join(f"{k} {extra['learned_3d'][k]['ms_per_step']:.1f} ms/step"
                                         for k in ("plain_fp64", "mixed", "mixed_learned")))
        if not args.no_upscaling:
            log("upscaling run (micromodel, to +20 % porosity)")
            extra["upscaling"] = upscaling_leg(vos, inputs, scaling, args.upscaling_budget, 0.2, args.dt)
            u = extra["upscaling"]
            log(f"upscaling: {u['steps']} steps in {u['wall_s']} s, phi {u['phi_start']:.4f} -> {u['phi_end']:.4f}")
        if not args.no_micromodel:
            log("micromodel 1024x512")
            extra["micromodel_mall_resident"] = micromodel_leg(vos, inputs, scaling, 20, 3, args.dt)
        if not args.no_micromodel_sweep:
            log("micromodel runs: Pe x Da x precision, 200 steps each")
            extra["micromodel_sweep"] = micromodel_sweep(vos, inputs, scaling, 200, args.dt)
            for r in extra["micromodel_sweep"]["runs"]:
                log(f"  Pe {r['Pe']:g} Da {r['Da']:g} {r['precision']}: {r['ms_per_step']:.3f} ms/step")
        if not args.no_batch:
            log(f"batch of {args.batch_n} micromodels")
            extra["batch_micromodels"] = batch_bench(vos, inputs, scaling, args.batch_n, args.batch_steps, args.dt)
        if not args.no_unet:
            log(f"U-Net {args.unet_n}^3")
            extra["unet"] = unet_bench(inputs, args.unet_n, 2)
        extra["hbm_streaming_ceiling"] = streaming_ceiling()
    cpu = None
    if not args.no_cpu_baseline and not args.only_headline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline_pack(args.cpu_crop, params, args.dt, args.cpu_budget)
    out = {
        "metric": "cell-steps/s + pressure-solve HBM GB/s at 1e-8 residual; learned+mixed vs plain",
        "value": head["value"],
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (FP32 multigrid preconditioners)",
        "data": "synthetic",
        "config": {"workload": f"grain pack {n}^3 dx=4um, log-normal spheres (median 20 voxels, sigma 0.3) "
                               f"seed 33 to porosity 0.23, 1% interface noise, constant-pressure drive at "
                               f"Pe={args.pe:g}, Da={args.da:g}, iVoS, dt={args.dt:g}s, dissolving, rtol 1e-8",
                   "precision": "mixed", "cells": cells,
                   "solver_starts": {0: "x^n", 1: "extrapolated 2x^n - x^(n-1)",
                                     2: "extrapolated 2x^n - x^(n-1) or 3x^n - 3x^(n-1) + x^(n-2), "
                                        "the order that predicted x^n better"}[EXTRAPOLATE],
                   "multigrid_setup_every_steps": SETUP_EVERY,
                   "setup": {"K": info["K"], "phi_without_bands": info["phi"], "dp_Pa": info["dp"],
                             "kc": info["kc"]}},
        "pressure_solve": {"GBs_algorithmic": head["pressure_GBs_algorithmic"],
                           "frac_hbm": head["pressure_frac_hbm"],
                           "its_per_step": head["pressure_its_per_step"],
                           "its_fp64_hierarchy_per_step": head["pressure_its_fp64_hierarchy"],
                           "ms_per_step": head["pressure_ms_per_step"]},
        "headline_run": head,
        "plain_fp64": comps.get("plain_fp64"),
        "psi_prime_mixed": comps.get("psi_prime_mixed"),
        "roofline": roof,
        "roofline_other_kernels": others,
        "cpu_baseline": cpu,
    }
    out.update(extra)
    if args.trace_window:
        os.makedirs(os.path.dirname(os.path.abspath(args.trace_window)), exist_ok=True)
        with open(args.trace_window, "w") as f:
            json.dump(TRACE_WINDOWS, f)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
