"""The C-ABI library builds for gfx950, loads, and exports every entry point
the headers under include/ declare (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for h in sorted(os.listdir(inc)):
        if h.endswith(".h"):
            src = re.sub(r"/\*.*?\*/", "", open(os.path.join(inc, h)).read(), flags=re.S)
            names |= set(re.findall(r"\b(vos_[a-z_]+)\s*\(", src))
    return sorted(names)


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("vos_create", "vos_step", "vos_set_solid_fraction", "vos_get_field",
                 "vos_workspace_bytes", "vos_destroy", "vos_last_error", "vos_diagnostics"):
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2204_07019_amd import vos
    if not os.path.exists(vos.LIB_PATH):
        from paper_2204_07019_amd import build
        build.build()
    lib = ctypes.CDLL(vos.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_argument_errors_without_a_device():
    """Host-side validation runs before any device call."""
    from paper_2204_07019_amd import vos
    L = vos.lib()
    g = vos._Grid(1, 4, 1, 1e-6)
    o = vos._Opts(**vos.asdict(vos.Opts()))
    n = ctypes.c_size_t()
    assert L.vos_workspace_bytes(ctypes.byref(g), ctypes.byref(o), ctypes.byref(n)) == vos.VOS_ERR_ARG
    assert b"nx >= 2" in L.vos_last_error()
    g = vos._Grid(64, 32, 1, 5e-6)
    assert L.vos_workspace_bytes(ctypes.byref(g), ctypes.byref(o), ctypes.byref(n)) == vos.VOS_OK
    assert n.value > 64 * 32 * 8 * 20
    for field, value in (("mg_nu", 9), ("level_kernels", 2), ("p_fp32_its", -1), ("extrapolate", 3), ("setup_every", -1),
                         ("deps_max", -1.0), ("deps_max", float("nan"))):
        bad = vos._Opts(**dict(vos.asdict(vos.Opts()), **{field: value}))
        assert L.vos_workspace_bytes(ctypes.byref(g), ctypes.byref(bad), ctypes.byref(n)) == vos.VOS_ERR_ARG, field
        assert field.encode() in L.vos_last_error()
    mixed = vos._Opts(**dict(vos.asdict(vos.Opts()), precision=vos.MIXED))
    m = ctypes.c_size_t()
    assert L.vos_workspace_bytes(ctypes.byref(g), ctypes.byref(mixed), ctypes.byref(m)) == vos.VOS_OK


def test_unet_host_validation_without_a_device():
    from paper_2204_07019_amd import unet
    assert unet.param_count() == 359761
    L = unet.lib()
    n = ctypes.c_size_t()
    for bad in [(1, 8, 8, 48, 4, 1), (1, 6, 8, 64, 4, 1), (1, 8, 8, 64, 0, 1), (1, 8, 8, 64, 17, 1),
                (0, 8, 8, 64, 4, 1)]:
        s = unet._Shape(*bad)
        assert L.vos_unet_workspace_bytes(ctypes.byref(s), ctypes.byref(n)) == 1, bad
    s = unet._Shape(2, 8, 8, 64, 4, 1)
    assert L.vos_unet_workspace_bytes(ctypes.byref(s), ctypes.byref(n)) == 0
    train = n.value
    s = unet._Shape(2, 8, 8, 64, 4, 0)
    assert L.vos_unet_workspace_bytes(ctypes.byref(s), ctypes.byref(n)) == 0
    assert 0 < n.value < train
    # activations: >= 224 bytes per full-resolution voxel for inference
    assert n.value >= 2 * 8 * 8 * 64 * 224
