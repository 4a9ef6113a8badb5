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
                 "vos_workspace_bytes", "vos_destroy", "vos_last_error", "vos_diagnostics",
                 "vos_solve_pressure", "vos_initialize", "vos_state_bytes", "vos_get_state", "vos_set_state",
                 "vos_solve_pressure_noalloc", "vos_unet_save", "vos_unet_load"):
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
    bad = vos._Opts(**dict(vos.asdict(vos.Opts()), solid_dt=-1.0))
    assert L.vos_workspace_bytes(ctypes.byref(g), ctypes.byref(bad), ctypes.byref(n)) == vos.VOS_ERR_ARG
    assert b"solid_dt" in L.vos_last_error()
    # the SIMPLE loop's options are checked when it is on
    for field, value in (("relax_u", 0.0), ("relax_p", 1.5), ("relax_c", -1.0), ("outer_max", 0),
                         ("outer_tol", -1.0), ("extrapolate", 1)):
        bad = vos._Opts(**dict(vos.asdict(vos.Opts()), simple=1, **{field: value}))
        assert L.vos_workspace_bytes(ctypes.byref(g), ctypes.byref(bad), ctypes.byref(n)) == vos.VOS_ERR_ARG, field
    ok = vos._Opts(**dict(vos.asdict(vos.Opts()), simple=1))
    assert L.vos_workspace_bytes(ctypes.byref(g), ctypes.byref(ok), ctypes.byref(n)) == vos.VOS_OK
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


def test_noalloc_pressure_validates_on_the_host():
    """The no-allocation pressure solve checks its arguments and the scratch
    limit (48 MiB) before touching a device."""
    from paper_2204_07019_amd import inputs, vos
    L = vos.lib()
    o = vos._Opts(**vos.asdict(vos.Opts()))
    pr = vos.make_params(dict(inputs.BASE_PARAMS, model=0))
    dummy = ctypes.c_void_p(256)
    big = vos._Grid(600, 400, 1, 5e-6)
    rc = L.vos_solve_pressure_noalloc(ctypes.byref(big), ctypes.byref(pr), ctypes.byref(o), 1e-3, dummy, dummy, dummy,
                                      None, dummy, None, None)
    assert rc == vos.VOS_ERR_ARG and b"scratch" in L.vos_last_error()
    g = vos._Grid(64, 32, 1, 5e-6)
    rc = L.vos_solve_pressure_noalloc(ctypes.byref(g), ctypes.byref(pr), ctypes.byref(o), 1e-3, None, dummy, dummy,
                                      None, dummy, None, None)
    assert rc == vos.VOS_ERR_ARG and b"NULL" in L.vos_last_error()
    tr = vos.make_params(dict(inputs.BASE_PARAMS, model=0, transient=1))
    rc = L.vos_solve_pressure_noalloc(ctypes.byref(g), ctypes.byref(tr), ctypes.byref(o), 1e-3, dummy, dummy, dummy,
                                      None, dummy, None, None)
    assert rc == vos.VOS_ERR_ARG and b"source" in L.vos_last_error()


def test_parameter_combinations_rejected():
    """Variant combinations the library refuses (as the oracle does)."""
    from paper_2204_07019_amd import inputs, vos
    L = vos.lib()
    g = vos._Grid(16, 8, 1, 5e-6)
    o = vos._Opts(**vos.asdict(vos.Opts()))
    ws = ctypes.c_void_p(256)
    h = ctypes.c_void_p()
    for kw in (dict(model=0, grad_scheme=1), dict(model=2, psi_kind=1), dict(model=0, drive=2),
               dict(model=0, Vm_f=-1.0)):
        pr = vos.make_params(dict(inputs.BASE_PARAMS, **kw))
        rc = L.vos_create(ctypes.byref(g), ctypes.byref(pr), ctypes.byref(o), ws, 1 << 40, None, ctypes.byref(h))
        assert rc == vos.VOS_ERR_ARG, kw
    # a separate solid step does not go with the transient storage terms
    pr = vos.make_params(dict(inputs.BASE_PARAMS, model=0, transient=1))
    os_ = vos._Opts(**dict(vos.asdict(vos.Opts()), solid_dt=1.0))
    rc = L.vos_create(ctypes.byref(g), ctypes.byref(pr), ctypes.byref(os_), ws, 1 << 40, None, ctypes.byref(h))
    assert rc == vos.VOS_ERR_ARG and b"solid_dt" in L.vos_last_error()
