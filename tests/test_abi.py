"""The C ABI library loads, exports every declared symbol, and rejects bad
arguments on the host before touching a GPU (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "mmx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(\w+)\s*\(", src, flags=re.M)))


def test_header_declarations_are_exported():
    from paper_2606_01114_amd import _lib
    L = _lib.lib()
    names = _declared()
    assert len(names) >= 19
    for n in names:
        assert hasattr(L, n), n
    assert sorted(_lib.EXPORTS) == names


def test_strerror():
    from paper_2606_01114_amd import _lib
    L = _lib.lib()
    assert L.mm_strerror(0) == b"ok"
    assert L.mm_strerror(-1) == b"invalid argument"
    assert L.mm_strerror(-99) == b"unknown status"


def _init(grid, cell, prec=1, opts=None):
    from paper_2606_01114_amd import _lib
    L = _lib.lib()
    h = ctypes.c_void_p()
    g = (ctypes.c_int64 * 3)(*grid)
    c = (ctypes.c_double * 3)(*cell)
    return L.demag_tensor_init(ctypes.byref(h), g, c, prec, None, opts), h


@pytest.mark.parametrize("grid,cell,prec", [
    ((0, 4, 4), (1e-9, 1e-9, 1e-9), 1),
    ((4, -1, 4), (1e-9, 1e-9, 1e-9), 1),
    ((4, 4, 4), (1e-9, 0.0, 1e-9), 1),
    ((4, 4, 4), (1e-9, float("nan"), 1e-9), 1),
    ((4, 4, 4), (1e-9, 1e-9, 1e-9), 3),
])
def test_init_rejects_bad_arguments(grid, cell, prec):
    from paper_2606_01114_amd import _lib
    rc, h = _init(grid, cell, prec)
    assert rc == _lib.MM_EINVAL and not h.value
    assert len(_lib.lib().mm_last_error()) > 0


def test_init_rejects_bad_padding():
    from paper_2606_01114_amd import _lib
    o = _lib.PlanOpts()
    assert _lib.lib().mm_plan_opts_default(ctypes.byref(o)) == 0
    assert o.far_radius == 16.0
    o.L[0] = 11                                   # 11 is not 7-smooth
    rc, _ = _init((4, 4, 4), (1e-9, 1e-9, 1e-9), 1, ctypes.byref(o))
    assert rc == _lib.MM_EINVAL
    o.L[0] = 6                                    # < 2n - 1
    rc, _ = _init((4, 4, 4), (1e-9, 1e-9, 1e-9), 1, ctypes.byref(o))
    assert rc == _lib.MM_EINVAL
    o.L[0] = 0
    o.autotune = 7
    rc, _ = _init((4, 4, 4), (1e-9, 1e-9, 1e-9), 1, ctypes.byref(o))
    assert rc == _lib.MM_EINVAL


def test_calls_on_null_plan():
    from paper_2606_01114_amd import _lib
    L = _lib.lib()
    dummy = ctypes.c_void_p(16)
    assert L.h_eff(None, dummy, None, 8e5, 1e-11, dummy, 3, None) == _lib.MM_EINVAL
    assert L.llg_step(None, dummy, None, 8e5, 1e-11, 0.1, 2.2e5, 1e-13, 1, None, 0) == _lib.MM_EINVAL
    assert L.h_eff_adjoint(None, dummy, None, 8e5, 1e-11, dummy, dummy, None, 3) == _lib.MM_EINVAL
    assert L.mm_plan_destroy(None) == _lib.MM_EINVAL
    assert L.mm_batch_destroy(None) == _lib.MM_EINVAL
    h = ctypes.c_void_p()
    assert L.mm_batch_create(ctypes.byref(h), 0, None, None, 1, None, None) == _lib.MM_EINVAL


def test_no_gpu_is_a_hip_error():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2606_01114_amd import _lib
    rc, h = _init((4, 4, 2), (1e-9, 1e-9, 1e-9), 1)
    assert rc == _lib.MM_EHIP and not h.value


def test_strerror_nonfinite():
    from paper_2606_01114_amd import _lib
    assert _lib.lib().mm_strerror(_lib.MM_ENONFINITE) == b"non-finite result"


def _bytes(grid, prec, opts=None):
    from paper_2606_01114_amd import _lib
    t, w = ctypes.c_size_t(), ctypes.c_size_t()
    g = (ctypes.c_int64 * 3)(*grid)
    rc = _lib.lib().mm_plan_bytes(g, prec, opts, ctypes.byref(t), ctypes.byref(w))
    return rc, t.value, w.value


def test_plan_bytes_host_only():
    """mm_plan_bytes needs no GPU: the tensor octant and the forward
    workspace of the 1024x1024x128 grid (padded 2048x2048x256)."""
    from paper_2606_01114_amd import _lib
    n, L = (1024, 1024, 128), (2048, 2048, 256)
    hx, hy, hz = L[0] // 2 + 1, L[1] // 2 + 1, L[2] // 2 + 1
    for prec, r in ((_lib.MM_F32, 4), (_lib.MM_F64, 8)):
        rc, t, w = _bytes(n, prec)
        assert rc == _lib.MM_OK
        assert t == hx * hy * hz * 6 * r
        c = 2 * r
        s1 = hz * n[0] * n[1] * 3 * c
        s2 = hz * L[0] * n[1] * 3 * c
        cells3 = n[0] * n[1] * n[2] * 3 * r
        big = s1 + s2 + 3 * cells3
        assert big <= w <= big + (64 << 20), (w, big)
    # explicit padding changes the sizes the same way plan creation does
    o = _lib.PlanOpts()
    _lib.lib().mm_plan_opts_default(ctypes.byref(o))
    o.pow2_padding = 1
    rc, t, _ = _bytes((48, 20, 3), _lib.MM_F32, ctypes.byref(o))
    assert rc == 0 and t == (128 // 2 + 1) * (64 // 2 + 1) * (8 // 2 + 1) * 6 * 4
    g = (ctypes.c_int64 * 3)(4, 4, 4)
    assert _lib.lib().mm_plan_bytes(g, 1, None, None, None) == _lib.MM_EINVAL
    assert _bytes((0, 4, 4), 1)[0] == _lib.MM_EINVAL
    assert _bytes((4, 4, 4), 5)[0] == _lib.MM_EINVAL


def test_bench_pass_bytes_against_plan_bytes_non_square():
    """The benchmark's byte model uses the spectrum sizes the library
    allocates: S1 = 3 nx ny hz and S2 = 3 Lx ny hz complex values (a
    non-square grid, so that nx, ny and Lx, Ly differ), plus the three
    stage fields, within the small tables of the workspace."""
    import bench
    from paper_2606_01114_amd import _lib
    n = (96, 40, 6)
    o = _lib.PlanOpts()
    _lib.lib().mm_plan_opts_default(ctypes.byref(o))
    o.pow2_padding = 1
    L = (256, 128, 16)
    hx, hy, hz = L[0] // 2 + 1, L[1] // 2 + 1, L[2] // 2 + 1
    for prec, r in ((_lib.MM_F32, 4), (_lib.MM_F64, 8)):
        rc, t, w = _bytes(n, prec, ctypes.byref(o))
        assert rc == 0
        b, _ = bench.pass_bytes(n, L, r)
        c = 2 * r
        S1, S2 = 3 * n[0] * n[1] * hz, 3 * L[0] * n[1] * hz
        T6 = 6 * hx * hy * hz
        assert b["x_fwd"] == c * (S1 + S2) and b["y_fused"] == 2 * c * S2 + r * T6
        assert t == r * T6
        big = c * (S1 + S2) + 3 * 3 * n[0] * n[1] * n[2] * r
        assert big <= w <= big + (1 << 20), (w, big)


def test_scratch_bytes_host_only():
    """mm_plan_scratch_bytes: 14 vector fields for the adjoint, 7 for RKF45,
    3 plus block sums for the minimiser (no GPU call)."""
    from paper_2606_01114_amd import _lib
    n = (1024, 1024, 128)
    for prec, r in ((_lib.MM_F32, 4), (_lib.MM_F64, 8)):
        out = (ctypes.c_size_t * 3)()
        g = (ctypes.c_int64 * 3)(*n)
        assert _lib.lib().mm_plan_scratch_bytes(g, prec, None, out) == 0
        f3 = n[0] * n[1] * n[2] * 3 * r
        assert out[0] == 14 * f3 and out[1] == 7 * f3
        assert 3 * f3 < out[2] < 3 * f3 + (16 << 20)
    g = (ctypes.c_int64 * 3)(4, 4, 4)
    assert _lib.lib().mm_plan_scratch_bytes(g, 1, None, None) == _lib.MM_EINVAL


def test_attach_on_null_plan():
    from paper_2606_01114_amd import _lib
    dummy = ctypes.c_void_p(256)
    assert _lib.lib().mm_plan_attach_memory(None, dummy, dummy) == _lib.MM_EINVAL
    assert _lib.lib().mm_plan_attach_scratch(None, dummy, 256) == _lib.MM_EINVAL
    assert _lib.lib().mm_batch_tensor_set(None, 0, None) == _lib.MM_EINVAL


def test_rkf45_rejects_bad_arguments_on_host():
    from paper_2606_01114_amd import _lib
    L = _lib.lib()
    dummy = ctypes.c_void_p(256)
    dt, err, ok = ctypes.c_double(1e-13), ctypes.c_double(), ctypes.c_int()
    assert L.llg_rkf45_step(None, dummy, None, 8e5, 1e-11, 0.1, 2.2e5, ctypes.byref(dt), 1e-5, None, 0,
                            ctypes.byref(err), ctypes.byref(ok)) == _lib.MM_EINVAL


def test_minimize_rejects_bad_arguments_on_host():
    from paper_2606_01114_amd import _lib
    L = _lib.lib()
    dummy = ctypes.c_void_p(256)
    it, tq = ctypes.c_int(), ctypes.c_double()
    assert L.mm_minimize_bb(None, dummy, None, 8e5, 1e-11, None, 1.0, 10, ctypes.byref(it),
                            ctypes.byref(tq)) == _lib.MM_EINVAL


def test_set_dmi_rejects_bad_arguments_on_host():
    from paper_2606_01114_amd import _lib
    L = _lib.lib()
    assert L.mm_plan_set_dmi(None, 1, 1e-3) == _lib.MM_EINVAL


def test_set_anisotropy_rejects_bad_arguments_on_host():
    from paper_2606_01114_amd import _lib
    L = _lib.lib()
    ax = (ctypes.c_double * 3)(0.0, 0.0, 1.0)
    assert L.mm_plan_set_anisotropy(None, 1e5, ax) == _lib.MM_EINVAL


def test_set_stt_rejects_bad_arguments_on_host():
    from paper_2606_01114_amd import _lib
    L = _lib.lib()
    pv = (ctypes.c_double * 3)(0.0, 0.0, 1.0)
    assert L.mm_plan_set_stt(None, 1e11, 0.4, 1.0, 0.0, 1e-9, pv) == _lib.MM_EINVAL


def test_longest_y_lines_on_host():
    """An FP64 y line of 4096 points (whose whole three-component pencil
    would need 209 KB of LDS) is planned as two half-spectra of 2048 points;
    y lines of 8192 points are refused in either precision (no GPU)."""
    from paper_2606_01114_amd import _lib
    o = _lib.PlanOpts()
    _lib.lib().mm_plan_opts_default(ctypes.byref(o))
    o.pow2_padding = 1
    for prec in (_lib.MM_F32, _lib.MM_F64):
        rc, t, _ = _bytes((4, 2048, 3), prec, ctypes.byref(o))
        assert rc == _lib.MM_OK and t == 5 * 2049 * 5 * 6 * (4 if prec == _lib.MM_F32 else 8)
        assert _bytes((4, 4096, 3), prec, ctypes.byref(o))[0] == _lib.MM_ENOTSUP


def test_automatic_padding_on_host():
    """The default padding takes the shortest compile-time length (powers of
    two: x, y 4096, z and an FP64 y 2048; one odd radix: x, y 96 ... 1792,
    z 96 ... 896) when it is at most 1.75 times the 7-smooth length; 0 keeps the
    7-smooth lengths, 1 powers of two, 3 the compile-time lengths
    unconditionally."""
    from paper_2606_01114_amd import _lib

    def tensor_L(grid, prec, pad=None):
        o = None
        if pad is not None:
            o = _lib.PlanOpts()
            _lib.lib().mm_plan_opts_default(ctypes.byref(o))
            o.pow2_padding = pad
            o = ctypes.byref(o)
        rc, t, _ = _bytes(grid, prec, o)
        assert rc == _lib.MM_OK
        return t

    def octant(L, r):
        return (L[0] // 2 + 1) * (L[1] // 2 + 1) * (L[2] // 2 + 1) * 6 * r

    F32, F64 = _lib.MM_F32, _lib.MM_F64
    assert tensor_L((350, 350, 350), F64) == octant((768, 768, 768), 8)
    assert tensor_L((350, 350, 350), F64, 0) == octant((700, 700, 700), 8)
    assert tensor_L((350, 350, 350), F64, 1) == octant((1024, 1024, 1024), 8)
    assert tensor_L((300, 6, 2), F32) == octant((640, 16, 4), 4)
    assert tensor_L((260, 6, 2), F32) == octant((640, 16, 4), 4)
    assert tensor_L((330, 6, 2), F32) == octant((768, 16, 4), 4)
    assert tensor_L((150, 180, 3), F32) == octant((320, 384, 8), 4)
    assert tensor_L((100, 220, 3), F64) == octant((224, 448, 8), 8)
    assert tensor_L((400, 5, 400), F32) == octant((896, 16, 896), 4)
    assert tensor_L((700, 5, 400), F32) == octant((1536, 16, 896), 4)
    assert tensor_L((160, 160, 160), F64) == octant((320, 320, 320), 8)
    assert tensor_L((5, 5, 500), F32) == octant((16, 16, 1024), 4)
    assert tensor_L((850, 640, 3), F32) == octant((1792, 1280, 8), 4)
    assert tensor_L((4, 1500, 1100), F32) == octant((8, 4096, 2205), 4)
    assert tensor_L((4, 4, 700), F32) == octant((8, 8, 2048), 4)
    assert tensor_L((4, 1500, 3), F64) == octant((8, 3000, 8), 8)
    assert tensor_L((4, 1100, 3), F32, 3) == octant((8, 4096, 8), 4)
    assert tensor_L((4, 4, 700), F32, 3) == octant((8, 8, 2048), 4)
    assert tensor_L((4, 4, 1500), F32, 3) == octant((8, 8, 4096), 4)   # past the compile-time z lengths
    o = _lib.PlanOpts()
    _lib.lib().mm_plan_opts_default(ctypes.byref(o))
    assert o.pow2_padding == 2
    o.pow2_padding = 4
    assert _bytes((4, 4, 4), F32, ctypes.byref(o))[0] == _lib.MM_EINVAL


def test_llg_stability_bound():
    """The host-side stiffness bound (no GPU): gamma (2A/(mu0 Ms)) sum 4/d^2
    dt -- 0.99 for the 2.5x2.5x3 nm film at Ms 8e5, 1.97 at Ms 4e5, and a 2 nm
    cube at Ms 4e5 past RK4's limit -- and its argument checks; the binding
    warns once for an unstable scalar-Ms configuration."""
    import math
    import warnings
    from paper_2606_01114_amd import RK4_IMAG_LIMIT, llg_stability
    from paper_2606_01114_amd import api
    from paper_2606_01114_amd._lib import MM_EINVAL, MMError
    mu0 = 4e-7 * math.pi
    d = (2.5e-9, 2.5e-9, 3e-9)
    for Ms in (8e5, 4e5):
        w = llg_stability(d, Ms, 1.3e-11, 2.211e5, 1e-13)
        ref = 2.211e5 * (2 * 1.3e-11 / (mu0 * Ms)) * sum(4 / v ** 2 for v in d) * 1e-13
        assert abs(w - ref) <= 1e-12 * ref
    assert llg_stability(d, 8e5, 1.3e-11, 2.211e5, 1e-13) < 1.0 < llg_stability(d, 4e5, 1.3e-11, 2.211e5, 1e-13) < 2.0
    assert llg_stability((2e-9,) * 3, 4e5, 1.3e-11, 2.211e5, 1e-13) > RK4_IMAG_LIMIT
    for bad in [((0.0, 1e-9, 1e-9), 8e5, 1e-13), (d, 0.0, 1e-13), (d, 8e5, -1e-13), (d, float("nan"), 1e-13)]:
        with pytest.raises(MMError) as ei:
            llg_stability(bad[0], bad[1], 1.3e-11, 2.211e5, bad[2])
        assert ei.value.code == MM_EINVAL
    with warnings.catch_warnings(record=True) as rec:
        warnings.simplefilter("always")
        api._stability_warning((2e-9,) * 3, 4e5, 1.3e-11, 2.211e5, 1e-13)
        api._stability_warning((2e-9,) * 3, 4e5, 1.3e-11, 2.211e5, 1e-13)
        api._stability_warning(d, 8e5, 1.3e-11, 2.211e5, 1e-13)
    assert len(rec) == 1 and "stability" in str(rec[0].message)


def test_bench_padding_table_matches_library():
    """The benchmark's byte model pads a sweep geometry the way the library's
    padding mode 3 does: for every n up to 1100 on x and y and up to 700 on
    z, the length its table gives equals the one the library plans (read back
    from the tensor octant of an n x 1 x 1 grid)."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    from paper_2606_01114_amd import _lib
    o = _lib.PlanOpts()
    _lib.lib().mm_plan_opts_default(ctypes.byref(o))
    o.pow2_padding = 3
    for axis, top in ((0, 1100), (1, 1100), (2, 700)):
        for n in range(2, top):
            g = [1, 1, 1]
            g[axis] = n
            rc, t, _ = _bytes(tuple(g), _lib.MM_F32, ctypes.byref(o))
            assert rc == _lib.MM_OK
            Lh = t // (6 * 4)   # L/2 + 1 along the axis, 1 elsewhere
            assert 2 * (Lh - 1) == bench._ct_len(n, axis), (axis, n, 2 * (Lh - 1), bench._ct_len(n, axis))
