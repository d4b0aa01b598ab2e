"""Host-side checks of the C ABI (no GPU needed).

The library must load, export every function declared in include/cams.h,
and reject invalid arguments in cams_create before any device work.
"""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(cams_[a-z_0-9]+)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    from paper_1705_05783_amd import _cams
    if not os.path.exists(_cams.LIB_PATH):
        pytest.fail("libcams.so is not built (run __graft_entry__.build())")
    return _cams.load()


def test_every_declared_symbol_is_exported(lib):
    from paper_1705_05783_amd import _cams
    declared = _declared_functions()
    assert len(declared) >= 15
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(_cams.EXPORTED)


def _create(grid=None, fluid=None, opt=None):
    from paper_1705_05783_amd import _cams as C
    g = grid or C.cams_grid(16, 16, 8, 1.0, 1.0, 1.0, 4, 4, 4)
    f = fluid or C.cams_fluid(1.0, 0.1, 0.0, 1.0, 0.1)
    o = opt or C.cams_options(C.CAMS_R_FE, 0, 5, C.CAMS_FP64, 0, 1e-8, 100, 1e-8, 20)
    h = ctypes.c_void_p()
    s = C.cams_create(ctypes.byref(g), ctypes.byref(f), ctypes.byref(o), None, ctypes.byref(h))
    return s, h


def test_create_valid_makes_no_device_call(lib):
    from paper_1705_05783_amd import _cams as C
    s, h = _create()
    assert s == C.CAMS_OK
    assert C.cams_num_coarse(h) == 4 * 4 * 2
    nbytes = C.cams_workspace_bytes(h)
    assert nbytes > 16 * 16 * 8 * 8 * 25 and nbytes % 256 == 0
    # calls out of order are rejected on the host
    e = ctypes.c_double()
    assert C.cams_assemble(h, None, None, ctypes.byref(e)) == C.CAMS_E_STATE
    assert C.cams_build_basis(h) == C.CAMS_E_STATE
    assert C.cams_coarse_op(h) == C.CAMS_E_STATE
    assert C.cams_destroy(h) == C.CAMS_OK


@pytest.mark.parametrize("bad", [
    dict(nx=1), dict(rx=1), dict(rx=9), dict(rx=20), dict(nz=1, rz=2, bad2d=True),
    dict(nx=9, rx=2),  # last vertex one cell from the previous one
    dict(dx=0.0),
])
def test_create_rejects_bad_grids(lib, bad):
    from paper_1705_05783_amd import _cams as C
    kw = dict(nx=16, ny=16, nz=8, dx=1.0, dy=1.0, dz=1.0, rx=4, ry=4, rz=4)
    kw.update({k: v for k, v in bad.items() if k != "bad2d"})
    if bad.get("bad2d"):
        kw.update(nx=1)
    g = C.cams_grid(kw["nx"], kw["ny"], kw["nz"], kw["dx"], kw["dy"], kw["dz"], kw["rx"], kw["ry"], kw["rz"])
    s, h = _create(grid=g)
    assert s == C.CAMS_E_ARG and not h.value


@pytest.mark.parametrize("field,value", [("dt", 0.0), ("c", -1.0), ("mu", 0.0), ("rho0", -1.0)])
def test_create_rejects_bad_fluid(lib, field, value):
    from paper_1705_05783_amd import _cams as C
    f = C.cams_fluid(1.0, 0.1, 0.0, 1.0, 0.1)
    setattr(f, field, value)
    s, h = _create(fluid=f)
    assert s == C.CAMS_E_ARG


@pytest.mark.parametrize("field,value", [("restriction", 3), ("n_post", -1), ("n_pre", 65),
                                         ("lin_rtol", 0.0), ("lin_maxit", 0), ("newton_maxit", 0),
                                         ("precision", 7), ("smoother", 4), ("smoother", -1)])
def test_create_rejects_bad_options(lib, field, value):
    from paper_1705_05783_amd import _cams as C
    o = C.cams_options(C.CAMS_R_FE, 0, 5, C.CAMS_FP64, 0, 1e-8, 100, 1e-8, 20)
    setattr(o, field, value)
    s, h = _create(opt=o)
    assert s == C.CAMS_E_ARG


def test_two_dimensional_grid_accepted(lib):
    from paper_1705_05783_amd import _cams as C
    g = C.cams_grid(20, 20, 1, 1.0, 1.0, 1.0, 4, 4, 1)
    s, h = _create(grid=g)
    assert s == C.CAMS_OK
    assert C.cams_num_coarse(h) == 25
    C.cams_destroy(h)


def test_null_arguments(lib):
    from paper_1705_05783_amd import _cams as C
    assert C.cams_create(None, None, None, None, None) == C.CAMS_E_ARG
    assert C.cams_destroy(None) == C.CAMS_E_ARG
    assert C.cams_workspace_bytes(None) == 0


def test_learned_guard_arguments(lib):
    """The learned basis' global check takes a count >= 0 (0: off); no
    device call, so it runs without a GPU."""
    from paper_1705_05783_amd import _cams as C
    s, h = _create()
    assert s == C.CAMS_OK
    assert C.cams_set_learned_guard(h, 0) == C.CAMS_OK
    assert C.cams_set_learned_guard(h, 55) == C.CAMS_OK
    assert C.cams_set_learned_guard(h, -1) == C.CAMS_E_ARG
    assert C.cams_set_learned_guard(None, 5) == C.CAMS_E_ARG
    C.cams_destroy(h)


def test_mixed_precision_needs_block_smoother(lib):
    from paper_1705_05783_amd import _cams as C
    for prec in (C.CAMS_MIXED_FP32, C.CAMS_MIXED_BF16):
        o = C.cams_options(C.CAMS_R_FE, 0, 5, prec, C.CAMS_SMOOTH_BLOCK_ILU0, 1e-8, 100, 1e-8, 20)
        s, h = _create(opt=o)
        assert s == C.CAMS_OK
        n_mixed = C.cams_workspace_bytes(h)
        C.cams_destroy(h)
        for fp64_only in (C.CAMS_SMOOTH_RB_ILU0, C.CAMS_SMOOTH_NAT_ILU0):
            o.smoother = fp64_only
            s, h = _create(opt=o)
            assert s == C.CAMS_E_ARG
        o.smoother = 4                        # no such smoother
        s, h = _create(opt=o)
        assert s == C.CAMS_E_ARG
        o.smoother = C.CAMS_SMOOTH_BLOCK_ALT_ILU0
        s, h = _create(opt=o)
        assert s == C.CAMS_OK
        assert C.cams_workspace_bytes(h) > n_mixed   # the shifted grid's pivots (FP64 and FP32)
        C.cams_destroy(h)
    o = C.cams_options(C.CAMS_R_FE, 0, 5, C.CAMS_FP64, C.CAMS_SMOOTH_NAT_ILU0, 1e-8, 100, 1e-8, 20)
    s, h = _create(opt=o)
    assert s == C.CAMS_OK
    C.cams_destroy(h)
    o = C.cams_options(C.CAMS_R_FE, 0, 5, C.CAMS_FP64, 0, 1e-8, 100, 1e-8, 20)
    s, h = _create(opt=o)
    assert C.cams_workspace_bytes(h) < n_mixed
    C.cams_destroy(h)


def test_batch_create_validation(lib):
    """cams_batch_create checks its contexts on the host (no HIP call)."""
    from paper_1705_05783_amd import _cams as C

    def opts(**kw):
        o = C.cams_options(C.CAMS_R_FE, 0, 5, C.CAMS_MIXED_FP32, 0, 1e-8, 100, 1e-8, 1)
        for k, v in kw.items():
            setattr(o, k, v)
        return o

    ctxs = []
    for g in (C.cams_grid(16, 16, 8, 1.0, 1.0, 1.0, 4, 4, 4), C.cams_grid(20, 12, 9, 1.0, 1.0, 1.0, 5, 4, 3)):
        s, h = _create(grid=g, opt=opts())
        assert s == C.CAMS_OK
        ctxs.append(h)

    def create(hs):
        arr = (ctypes.c_void_p * len(hs))(*[h.value for h in hs])
        b = ctypes.c_void_p()
        return C.cams_batch_create(arr, len(hs), None, ctypes.byref(b)), b

    s, b = create(ctxs)
    assert s == C.CAMS_OK
    assert C.cams_batch_workspace_bytes(b) % 256 == 0 and C.cams_batch_workspace_bytes(b) > 0
    # before a workspace is attached, a solve is refused on the host
    assert C.cams_batch_newton_iteration(b, None, None, None, None) == C.CAMS_E_ARG
    C.cams_batch_destroy(b)
    s, b = create([ctxs[0], ctxs[0]])              # the same context twice
    assert s == C.CAMS_E_ARG
    s, h = _create(opt=opts(precision=C.CAMS_FP64))  # different precision
    s2, b = create([ctxs[0], h])
    assert s2 == C.CAMS_E_ARG
    C.cams_destroy(h)
    s, h = _create(opt=opts(n_post=3))             # different smoothing count
    s2, b = create([ctxs[0], h])
    assert s2 == C.CAMS_E_ARG
    C.cams_destroy(h)
    s, h = _create(opt=opts(precision=C.CAMS_FP64, smoother=C.CAMS_SMOOTH_RB_ILU0))
    s2, b = create([h])                              # red-black smoother is not batched
    assert s2 == C.CAMS_E_ARG
    C.cams_destroy(h)
    assert C.cams_batch_create(None, 0, None, ctypes.byref(ctypes.c_void_p())) == C.CAMS_E_ARG
    for h in ctxs:
        C.cams_destroy(h)


def test_coarse_layout_choice(lib):
    """Block-tridiagonal coarse factorisation exactly for 3D MSFE grids with
    more than 4096 coarse nodes and at least 3 coarse z-planes."""
    from paper_1705_05783_amd import _cams as C
    cases = [((256, 256, 128), C.CAMS_R_FE, 16), ((256, 256, 128), C.CAMS_R_FV, 0),
             ((128, 128, 128), C.CAMS_R_FE, 0),      # 4096 nodes: dense
             ((96, 96, 40), C.CAMS_R_FE, 10), ((200, 200, 16), C.CAMS_R_FE, 0)]   # 2 planes: dense
    for (nx, ny, nz), restr, planes in cases:
        r = 4 if (nx, ny, nz) == (96, 96, 40) else 8
        g = C.cams_grid(nx, ny, nz, 1.0, 1.0, 1.0, r, r, r)
        o = C.cams_options(restr, 0, 5, C.CAMS_FP64, 0, 1e-8, 100, 1e-8, 20)
        s, h = _create(grid=g, opt=o)
        assert s == C.CAMS_OK, (nx, ny, nz)
        assert C.cams_coarse_planes(h) == planes, ((nx, ny, nz), restr, C.cams_num_coarse(h))
        C.cams_destroy(h)
