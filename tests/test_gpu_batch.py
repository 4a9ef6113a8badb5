"""GPU tests of the batch API: instances of different sizes and parameters
advanced concurrently must be bit-identical to the same simulations run one
by one, before and after autotuning; a failing instance does not stop the
others."""
import numpy as np
import pytest

from paper_2204_07019_amd import inputs

pytestmark = pytest.mark.gpu

SIZES = [(64, 32), (96, 40), (128, 64), (40, 24), (64, 32)]
FIELDS = ("eps", "ux", "uy", "p", "c")


def specs():
    out = []
    rng = np.random.default_rng(3)
    for k, (nx, ny) in enumerate(SIZES):
        p = dict(inputs.BASE_PARAMS, model=k % 3)
        p["u_in"] = 1e-4 * 10 ** rng.uniform(-1, 1)
        p["kc"] = 1e-4 * 10 ** rng.uniform(-1, 0.5)
        out.append((nx, ny, 1, 5e-6, p))
    return out


def geometry(k, nx, ny):
    return inputs.rsa_discs(nx, ny, seed=40 + k, rmin=3, rmax=7, porosity=0.7)


def opts():
    from paper_2204_07019_amd import vos
    return vos.Opts(precision=vos.MIXED, rtol_u=1e-10, rtol_p=1e-10, rtol_c=1e-10)


def standalone(k, spec, steps, dt, start=None):
    from paper_2204_07019_amd import vos
    nx, ny, nz, dx, p = spec
    s = vos.Sim(nx, ny, nz, dx, p, opts())
    s.set_solid_fraction(geometry(k, nx, ny))
    if start is not None:
        for f, v in start.items():
            s.set(f, v)
    diags = [s.step(dt[k]) for _ in range(steps)]
    out = {f: s.get_numpy(f) for f in FIELDS}
    s.close()
    return out, diags


def test_batch_matches_standalone_bitwise():
    from paper_2204_07019_amd.batch import Batch
    print("batch of", len(SIZES), "vs standalone", flush=True)
    sp = specs()
    b = Batch(sp, opts(), workers=4)
    for k, (nx, ny, _, _, _) in enumerate(sp):
        b.sims[k].set_solid_fraction(geometry(k, nx, ny))
    dt = [1e-3 * (1 + 0.5 * k) for k in range(len(sp))]
    last = None
    for _ in range(3):
        last = b.step(dt)
    for k, s in enumerate(sp):
        ref, rd = standalone(k, s, 3, dt)
        for f in FIELDS:
            np.testing.assert_array_equal(b.sims[k].get_numpy(f), ref[f], err_msg=f"instance {k} {f}")
        assert last[k]["it_p"] == rd[-1]["it_p"] and last[k]["it_c"] == rd[-1]["it_c"]
    b.close()


def test_tuned_batch_still_bitwise():
    from paper_2204_07019_amd.batch import Batch
    print("batch tune", flush=True)
    sp = specs()
    b = Batch(sp, opts(), workers=2)
    for k, (nx, ny, _, _, _) in enumerate(sp):
        b.sims[k].set_solid_fraction(geometry(k, nx, ny))
    dt = [1e-3] * len(sp)
    b.step(dt, 2)
    t = b.tune(dt, probe_steps=1)
    print(t)
    assert 1 <= t["workers"] <= 16 and t["best_ms"] > 0
    # the chosen check intervals and tile shapes (the standalone references
    # below run with the defaults: every tile shape gives the same values)
    for k in range(len(sp)):
        tk = b.tuning(k)
        print(k, tk, flush=True)
        assert tk["check_every"] in (2, 4, 8, 16, 32) or tk["check_every"] == opts().check_every
        assert tk["tile_big_cells"] in (1 << 16, 1 << 18, 1 << 20, 0xFFFFFFFF)
    start = [{f: b.sims[k].get_numpy(f) for f in ("eps", "ux", "uy", "uz", "p", "c")} for k in range(len(sp))]
    b.step(dt, 2)
    for k, s in enumerate(sp):
        ref, _ = standalone(k, s, 2, dt, start=start[k])
        for f in FIELDS:
            np.testing.assert_array_equal(b.sims[k].get_numpy(f), ref[f], err_msg=f"instance {k} {f}")
    b.close()


def test_failing_instance_is_isolated():
    from paper_2204_07019_amd.batch import Batch
    from paper_2204_07019_amd import vos
    print("batch failure isolation", flush=True)
    sp = specs()[:3]
    b = Batch(sp, opts(), workers=3)
    for k, (nx, ny, _, _, _) in enumerate(sp):
        if k != 1:
            b.sims[k].set_solid_fraction(geometry(k, nx, ny))
    # instance 1 has no geometry: its step is out of order
    with pytest.raises(vos.VosError) as ei:
        b.step([1e-3] * 3)
    assert "instance 1" in str(ei.value)
    d = b.sims[0].diagnostics()
    assert d["it_p"] > 0 and b.sims[2].diagnostics()["it_p"] > 0
    b.close()


def test_batch_instance_matches_oracle(orc):
    """One instance of a concurrent batch (VoS-psi', the largest grid, mixed
    precision) against the FP64 oracle after 3 steps, at the 1e-6 bar."""
    from paper_2204_07019_amd import vos
    from paper_2204_07019_amd.batch import Batch
    from gpu_cases import make_problem, rel_l2
    sp = specs()
    tight = vos.Opts(precision=vos.MIXED, rtol_u=1e-12, rtol_p=1e-12, rtol_c=1e-12, maxit_p=20000)
    b = Batch(sp, tight, workers=4)
    for k, (nx, ny, _, _, _) in enumerate(sp):
        b.sims[k].set_solid_fraction(geometry(k, nx, ny))
    dt = [1e-3] * len(sp)
    k = 2   # 128 x 64, model 2
    print(f"batch of {len(sp)}; instance {k} against the oracle", flush=True)
    for _ in range(3):
        b.step(dt)
    g = {f: b.sims[k].get_numpy(f) for f in FIELDS}
    b.close()
    nx, ny, nz, dx, p = sp[k]
    es = geometry(k, nx, ny).reshape(1, ny, nx)
    prob = make_problem(es, dict(p, dx=dx), model=p["model"])
    st = orc.initial_state(prob, es)
    for _ in range(3):
        orc.step(prob, st, dt[k])
    err = {f: rel_l2(g[f], getattr(st, f)) for f in FIELDS}
    print("[parity] batch instance vs oracle:", {f: float(f"{v:.2e}") for f, v in err.items()}, flush=True)
    for f, v in err.items():
        assert v <= 1e-6, (f, v)
