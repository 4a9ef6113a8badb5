"""Every memory access of the z-marching kernels stays inside its array, on
the CPU: tests/emu/zmarch_emu.cpp runs the kernels' own source (vos_march3d.h
and the headers under it) once per block and thread of the library's launch
shapes, on every level of the pressure, transport and momentum hierarchies of
a grid, built with AddressSanitizer over one heap allocation per array.

Ragged grids and the 128^3 pack run by default; the 256^3 pack (about four
minutes) with VOS_EMU_FULL=1.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path_factory.mktemp("emu") / "zmarch_emu")
    cmd = ["g++", "-std=c++17", "-O2", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "tests", "emu"), "-I", os.path.join(ROOT, "paper_2204_07019_amd", "csrc"),
           os.path.join(ROOT, "tests", "emu", "zmarch_emu.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    return exe


def _run(exe, *dims, timeout=600):
    r = subprocess.run([exe, *map(str, dims)], capture_output=True, text=True, timeout=timeout)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "all in bounds" in r.stdout
    return r.stdout


def test_ragged_grids_in_bounds(emu):
    # widths around the tile (64 x 4), odd z, a grid narrower than half a tile
    out = _run(emu, 40, 33, 20, 97, 61, 45, 65, 5, 7, 31, 64, 9, 130, 7, 3)
    assert "transport FP64 level 0: 130 x 7 x 3" in out


def test_pack_128_in_bounds(emu):
    out = _run(emu, 128, 128, 128)
    assert "pressure FP32 level 0: 128 x 128 x 128" in out
    assert "momentum x FP64 level 0: 129 x 128 x 128" in out


def test_partly_filled_fused_launch_in_bounds(emu):
    # 144 FP64 tiles on 256 slots: the fused legs run short z-runs in several
    # rounds of blocks instead of one run per tile
    out = _run(emu, 384, 384, 32)
    assert "transport FP64 level 0: 384 x 384 x 32" in out


@pytest.mark.skipif(os.environ.get("VOS_EMU_FULL") != "1", reason="set VOS_EMU_FULL=1 (tens of minutes)")
def test_pack_256_in_bounds(emu):
    out = _run(emu, 256, 256, 256, timeout=1800)
    assert "pressure operator: z-run" in out
