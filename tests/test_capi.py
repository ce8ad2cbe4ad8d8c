"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/shape.h declares, and rejects bad arguments before
launching anything."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "shape.h")


@pytest.fixture(scope="module")
def shape():
    import paper_1203_0571_amd as shape
    return shape


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(shape_[a-z_0-9]+)\s*\(",
                                 text, flags=re.M)))


def test_header_declares_the_stage_calls():
    names = declared_functions()
    for f in ["shape_centroid", "shape_moments", "shape_fit_sersic", "shape_default_opts",
              "shape_status_string", "shape_abi_version"]:
        assert f in names


def test_library_exports_every_declared_symbol(shape):
    lib = C.CDLL(shape.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert shape.lib.shape_abi_version() == 2


def test_struct_layout_matches_header(shape):
    # offsets fixed by the header's field order on x86-64 / LP64
    assert C.sizeof(shape.ShapeBatch) == 6 * 8 + 8 + 8 + 4 + 4
    assert C.sizeof(shape.ShapeOpts) == 4 * 4 + 9 * 8 + 2 * 4 + 8


def test_defaults(shape):
    o = shape.default_opts()
    assert o.max_iter_centroid == 20 and o.max_iter_moments == 20 and o.max_iter_lm == 30
    assert o.k_gain == 0.75 and o.free_mask == 0xFF and o.gmax == 0.95
    assert o.tol_lm == 1e-5 and o.tol_sigma == 1e-4
    assert shape.lib.shape_default_opts(None) == shape.EINVAL


def test_status_strings(shape):
    for code in [0, -1, -2, -3, -4, 7]:
        assert isinstance(shape.lib.shape_status_string(code), bytes)


def _batch(shape, **kw):
    b = shape.ShapeBatch()
    b.pixels = 0x1000
    b.sigma = 0x2000
    b.n = 4
    b.n_pixels = 4 * 16 * 16
    b.side0 = 16
    b.dtype = shape.F32
    for k, v in kw.items():
        setattr(b, k, v)
    return b


def test_argument_errors_return_einval_without_launch(shape):
    L = shape.lib
    o = shape.default_opts()
    out = C.c_void_p(0x3000)
    cases = [
        _batch(shape, pixels=None),
        _batch(shape, sigma=None),
        _batch(shape, n=-1),
        _batch(shape, side0=3),
        _batch(shape, side0=129),
        _batch(shape, dtype=7),
        _batch(shape, dtype=shape.F16_SCALED),          # scale missing
        _batch(shape, n_pixels=3 * 16 * 16),            # uniform batch overruns the buffer
    ]
    for b in cases:
        assert L.shape_centroid(C.byref(b), C.byref(o), out, out, out, None) == shape.EINVAL
        assert L.shape_moments(C.byref(b), C.byref(o), out, out, out, out, None) == shape.EINVAL
        assert L.shape_fit_sersic(C.byref(b), C.byref(o), out, out, out, out, None, out, out,
                                  None, None) == shape.EINVAL
    b = _batch(shape)
    assert L.shape_centroid(None, C.byref(o), out, out, out, None) == shape.EINVAL
    assert L.shape_centroid(C.byref(b), None, out, out, out, None) == shape.EINVAL
    assert L.shape_centroid(C.byref(b), C.byref(o), None, out, out, None) == shape.EINVAL
    assert L.shape_fit_sersic(C.byref(b), C.byref(o), None, None, out, out, None, out, out,
                              None, None) == shape.EINVAL
    for field, val in [("k_gain", 0.0), ("gmax", 1.0), ("lambda0", -1.0), ("n0", 0.1),
                       ("max_iter_lm", -1), ("moffat_beta", 1.0), ("tol_sigma", -1.0)]:
        ob = shape.default_opts(**{field: val})
        assert L.shape_centroid(C.byref(b), C.byref(ob), out, out, out, None) == shape.EINVAL


def test_unsupported_mask_and_empty_batch(shape):
    L = shape.lib
    out = C.c_void_p(0x3000)
    b = _batch(shape)
    o = shape.default_opts(free_mask=0x0F)
    assert L.shape_fit_sersic(C.byref(b), C.byref(o), out, out, out, out, None, out, out,
                              None, None) == shape.EUNSUPPORTED
    e = _batch(shape, n=0, pixels=None, sigma=None)
    o = shape.default_opts()
    assert L.shape_centroid(C.byref(e), C.byref(o), None, None, None, None) == shape.OK
    assert L.shape_moments(C.byref(e), C.byref(o), None, None, None, None, None) == shape.OK
    assert L.shape_fit_sersic(C.byref(e), C.byref(o), None, None, None, None, None, None, None,
                              None, None) == shape.OK


def test_chi2_argument_errors(shape):
    L = shape.lib
    out = C.c_void_p(0x3000)
    b = _batch(shape)
    assert L.shape_chi2_fwd(C.byref(b), None, out, None) == shape.EINVAL
    assert L.shape_chi2_fwd(C.byref(b), out, None, None) == shape.EINVAL
    assert L.shape_chi2_bwd(C.byref(b), out, None, None, None, None, None, None) == shape.EINVAL
    bad = _batch(shape, side0=200)
    assert L.shape_chi2_fwd(C.byref(bad), out, out, None) == shape.EINVAL
    e = _batch(shape, n=0, pixels=None, sigma=None)
    assert L.shape_chi2_fwd(C.byref(e), None, None, None) == shape.OK
    assert L.shape_chi2_bwd(C.byref(e), None, None, None, None, None, None, None) == shape.OK
    assert L.shape_chi2_grad_scale(out, None, -1, out, None) == shape.EINVAL
    assert L.shape_chi2_grad_scale(None, None, 4, out, None) == shape.EINVAL
    assert L.shape_chi2_grad_scale(out, None, 4, None, None) == shape.EINVAL
    assert L.shape_chi2_grad_scale(None, None, 0, None, None) == shape.OK


def test_queue_argument_errors(shape):
    L = shape.lib
    out = C.c_void_p(0x3000)
    b = _batch(shape)
    o = shape.default_opts()
    c = shape.queue_cfg()
    assert c.team == 1 and c.grid == 0
    need = shape.queue_workspace_bytes(b.n)
    assert need >= b.n * 1000
    assert shape.queue_workspace_bytes(10 ** 6) > 400 * 10 ** 6
    nb = C.c_size_t()
    assert L.shape_queue_workspace_bytes(-1, C.byref(nb)) == shape.EINVAL
    # workspace too small
    assert L.shape_queue_start(C.byref(b), C.byref(o), C.byref(c), None, out, out, need - 1,
                               None) == shape.ENOMEM
    assert L.shape_queue_step(C.byref(b), C.byref(o), C.byref(c), out, need - 1, None) == shape.ENOMEM
    # missing workspace, missing starting point, bad team sizes
    assert L.shape_queue_step(C.byref(b), C.byref(o), C.byref(c), None, need, None) == shape.EINVAL
    assert L.shape_queue_start(C.byref(b), C.byref(o), C.byref(c), None, None, out, need,
                               None) == shape.EINVAL
    for team, side in [(3, 64), (2, 3), (4, 200), (0, 64)]:
        cc = shape.queue_cfg(team=team, team_min_side=side)
        assert L.shape_queue_step(C.byref(b), C.byref(o), C.byref(cc), out, need,
                                  None) == shape.EINVAL
    for chunk in (-1, 65):
        cc = shape.queue_cfg(chunk=chunk)
        assert L.shape_queue_step(C.byref(b), C.byref(o), C.byref(cc), out, need,
                                  None) == shape.EINVAL
    # the 4-parameter mask runs one wave per stamp only
    o4 = shape.default_opts(free_mask=0xF0)
    c2 = shape.queue_cfg(team=2, team_min_side=64)
    assert L.shape_queue_step(C.byref(b), C.byref(o4), C.byref(c2), out, need,
                              None) == shape.EUNSUPPORTED
    assert L.shape_queue_drain(C.byref(b), C.byref(o), C.byref(c), out, need - 1,
                               None) == shape.ENOMEM
    assert L.shape_queue_drain(C.byref(b), C.byref(o), None, out, need, None) == shape.EINVAL
    g = C.c_void_p()
    assert L.shape_queue_graph_create(C.byref(b), C.byref(o), C.byref(c), out, need - 1,
                                      C.byref(g)) == shape.ENOMEM
    assert L.shape_queue_graph_launch(None, None) == shape.EINVAL
    assert L.shape_queue_graph_destroy(None) == shape.EINVAL
    e = _batch(shape, n=0, pixels=None, sigma=None)
    assert L.shape_queue_step(C.byref(e), C.byref(o), C.byref(c), None, 0, None) == shape.OK


def test_static_queue_fit_limits(shape):
    """shape_fit_queue_static: more stamps than its static workspace holds is
    SHAPE_ENOMEM, checked before anything touches a device; bad arguments are
    SHAPE_EINVAL as for the other calls; an empty batch is a no-op."""
    L = shape.lib
    out = C.c_void_p(0x3000)
    o = shape.default_opts()
    c = shape.queue_cfg()
    assert shape.STATIC_MAX_STAMPS == 65536
    big = _batch(shape, n=shape.STATIC_MAX_STAMPS + 1, n_pixels=(shape.STATIC_MAX_STAMPS + 1) * 256)
    args = (None, out, out, out, None, out, out, None, None)
    assert L.shape_fit_queue_static(C.byref(big), C.byref(o), C.byref(c), *args) == shape.ENOMEM
    b = _batch(shape)
    assert L.shape_fit_queue_static(None, C.byref(o), C.byref(c), *args) == shape.EINVAL
    assert L.shape_fit_queue_static(C.byref(b), C.byref(o), None, *args) == shape.EINVAL
    assert L.shape_fit_queue_static(C.byref(b), C.byref(o), C.byref(c),
                                    None, None, out, out, None, out, out, None, None) == shape.EINVAL
    e = _batch(shape, n=0, pixels=None, sigma=None)
    assert L.shape_fit_queue_static(C.byref(e), C.byref(o), C.byref(c), *args) == shape.OK


def test_star_moments_argument_errors(shape):
    L = shape.lib
    out = C.c_void_p(0x3000)
    b = _batch(shape)
    assert L.shape_star_moments(C.byref(b), 2, out, 1e-4, 20, out, out, out, None) == shape.EINVAL
    assert L.shape_star_moments(C.byref(b), 0, out, -1.0, 20, out, out, out, None) == shape.EINVAL
    assert L.shape_star_moments(C.byref(b), 0, out, 1e-4, -1, out, out, out, None) == shape.EINVAL
    assert L.shape_star_moments(C.byref(b), 1, None, 1e-4, 20, out, out, out, None) == shape.EINVAL
    assert L.shape_star_moments(C.byref(b), 1, out, 1e-4, 20, out, None, out, None) == shape.EINVAL
    assert L.shape_star_moments(None, 1, out, 1e-4, 20, out, out, out, None) == shape.EINVAL
    e = _batch(shape, n=0, pixels=None, sigma=None)
    assert L.shape_star_moments(C.byref(e), 0, None, 1e-4, 20, None, None, None, None) == shape.OK
    Lb = L.shape_star_moments_beta
    for beta in (1.0, 0.5, -3.0, float("nan"), 2e6):
        assert Lb(C.byref(b), beta, out, 1e-4, 20, out, out, out, None) == shape.EINVAL
    assert Lb(C.byref(b), 3.0, out, -1.0, 20, out, out, out, None) == shape.EINVAL
    assert Lb(C.byref(b), 3.0, out, 1e-4, -1, out, out, out, None) == shape.EINVAL
    assert Lb(C.byref(b), 3.0, None, 1e-4, 20, out, out, out, None) == shape.EINVAL
    assert Lb(None, 3.0, out, 1e-4, 20, out, out, out, None) == shape.EINVAL
    assert Lb(C.byref(e), 3.0, None, 1e-4, 20, None, None, None, None) == shape.OK


def _frames(shape, **kw):
    f = shape.ShapeFrames()
    f.pixels = 0x1000
    f.scale = None
    f.n = 3
    f.height = 64
    f.width = 80
    f.dtype = shape.F32
    for k, v in kw.items():
        setattr(f, k, v)
    return f


def test_frame_argument_errors(shape):
    L = shape.lib
    out = C.c_void_p(0x3000)
    assert C.sizeof(shape.ShapeFrames) == 2 * 8 + 8 + 4 * 4
    for bad in [dict(n=-1), dict(height=3), dict(width=4097), dict(dtype=7), dict(pixels=None),
                dict(dtype=shape.F16_SCALED)]:
        f = _frames(shape, **bad)
        assert L.shape_frame_detect(C.byref(f), 128, out, out, out, out, None) == shape.EINVAL
        assert L.shape_frame_cut(C.byref(f), out, out, out, 100, None, None) == shape.EINVAL
    f = _frames(shape)
    assert L.shape_frame_detect(None, 128, out, out, out, out, None) == shape.EINVAL
    for ms in (3, 129):
        assert L.shape_frame_detect(C.byref(f), ms, out, out, out, out, None) == shape.EINVAL
    assert L.shape_frame_detect(C.byref(f), 128, None, out, out, out, None) == shape.EINVAL
    assert L.shape_frame_detect(C.byref(f), 128, out, out, None, out, None) == shape.EINVAL
    assert L.shape_frame_cut(C.byref(f), None, out, out, 100, None, None) == shape.EINVAL
    assert L.shape_frame_cut(C.byref(f), out, out, None, 100, None, None) == shape.EINVAL
    assert L.shape_frame_cut(C.byref(f), out, out, out, -1, None, None) == shape.EINVAL
    assert L.shape_frame_offsets(out, -1, out, out, None) == shape.EINVAL
    assert L.shape_frame_offsets(out, 3, out, None, None) == shape.EINVAL
    assert L.shape_frame_offsets(None, 3, out, out, None) == shape.EINVAL
    e = _frames(shape, n=0, pixels=None)
    assert L.shape_frame_detect(C.byref(e), 128, None, None, None, None, None) == shape.OK
    assert L.shape_frame_cut(C.byref(e), None, None, None, 0, None, None) == shape.OK


def test_unprofiled_form_is_limited_to_the_4_parameter_sersic_fit(shape):
    L = shape.lib
    out = C.c_void_p(0x3000)
    b = _batch(shape)
    o = shape.default_opts(linear_init=0)          # all eight free: not provided
    assert L.shape_fit_sersic(C.byref(b), C.byref(o), out, None, out, out, None, out, out, None,
                              None) == shape.EUNSUPPORTED
    bm = _batch(shape, model=0x5000)
    o = shape.default_opts(linear_init=0, free_mask=shape.MASK_SIZE)
    assert L.shape_fit_sersic(C.byref(bm), C.byref(o), out, None, out, out, None, out, out, None,
                              None) == shape.EUNSUPPORTED
