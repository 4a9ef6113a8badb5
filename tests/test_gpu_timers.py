"""vos_time_kernel on a 3-D grid large enough for the fused finest-level legs
(>= 2^20 cells on the cell and x-face grids): every family either times its
launches (positive duration and bytes) or refuses with VOS_ERR_ARG (the 2-D
tiled legs), and the timed launches touch only scratch buffers -- the
simulation continues bitwise as an untouched twin does."""
import sys

import numpy as np
import pytest

from gpu_cases import gpu_sim, make_problem

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", [0, 1])
def test_timers_time_and_leave_the_state(orc, precision):
    from paper_2204_07019_amd import inputs, vos
    nx, ny, nz = 130, 64, 128
    rng = np.random.default_rng(17)
    es = np.clip(rng.uniform(-3.0, 1.5, (nz, ny, nx)), 0.0, 1.0)
    es[:, :, :2] = 0.0
    es[:, :, -2:] = 0.0
    prob = make_problem(es, dict(inputs.BASE_PARAMS, dx=5e-6), rtol_u=1e-9, rtol_p=1e-9, rtol_c=1e-9)
    sims = []
    for k in range(2):
        sim = gpu_sim(prob, precision)
        sim.set_solid_fraction(es)
        sim.step(1e-3)
        sims.append(sim)
    _say(f"timers {nx}x{ny}x{nz} precision {precision}")
    for fam, code in sorted(vos.KERNELS.items(), key=lambda kv: kv[1]):
        if fam in ("v_down", "v_up"):
            with pytest.raises(vos.VosError) as e:
                sims[0].time_kernel(fam, 2)
            assert e.value.status == vos.VOS_ERR_ARG
            continue
        t = sims[0].time_kernel(fam, 2)
        print(f"[timer] {fam}: {t['avg_ms'] * 1e3:.1f} us, {t['bytes'] / 1e6:.1f} MB", flush=True)
        assert t["avg_ms"] > 0 and t["bytes"] > 0, fam
    for sim in sims:
        sim.step(1e-3)
    for k in ("ux", "uy", "uz", "p", "c", "eps"):
        assert np.array_equal(sims[0].get_numpy(k), sims[1].get_numpy(k)), k
    for sim in sims:
        sim.close()
