"""The C ABI library: it loads without a GPU, exports every function that
include/hashpoint.h declares, and its host-side validation rejects bad
arguments before any launch (so these calls never touch a device)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2404_14044_amd import hashpoint as hp
from paper_2404_14044_amd import scenes

import oracle

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                      "include", "hashpoint.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hp_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_function():
    L = hp.lib()
    names = _declared()
    assert "hp_build_table" in names and "hp_render_backward" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(hp.EXPORTED)


def test_struct_sizes_match_header():
    # pointer-sized fields and int64 alignment as the C compiler lays them out
    assert ctypes.sizeof(hp.HPCamera) == 4 * 18
    assert ctypes.sizeof(hp.HPParams) == 4 * 27
    assert ctypes.sizeof(hp.HPViewInfo) == 32
    assert ctypes.sizeof(hp.HPSamples) == 8 * 9
    assert ctypes.sizeof(hp.HPMlp) == 8 * 6


def test_status_strings():
    L = hp.lib()
    for code in range(6):
        assert len(L.hp_status_str(code)) > 0
    assert L.hp_status_str(99) == b"unknown status"


def test_view_bounds_match_oracle_guard():
    for sc in (scenes.sphere_plane(n_sphere=10, n_plane=10), scenes.tiny_scene()):
        for inv in (0.0, 1.0 / sc.params.t_near):
            p = sc.params.replace(inv_tref=float(np.float32(inv)))
            g, d = hp.view_bounds(sc.cams[0], p)
            assert g == oracle.guard(sc.cams[0], p)
            assert g == int(np.floor(0.5 + d)) + 1 or abs(0.5 + d - round(0.5 + d)) < 1e-4


def test_workspace_size_grows_with_points():
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    a = hp.table_workspace(1000, sc.cams, sc.params)
    b = hp.table_workspace(100000, sc.cams, sc.params)
    assert b > a > 0


@pytest.mark.parametrize("field,value", [
    ("radius", 0.0), ("radius", float("nan")), ("t_near", 0.0), ("t_far", 0.5),
    ("K", 0), ("K", 33), ("n_samples", 0), ("n_samples", 65), ("m_cap", 0), ("m_cap", 65),
    ("gamma", 0.0), ("gamma", 1.5), ("eps_idw", 0.0), ("delta_last", 0.0), ("layout", 7),
    ("flags", 1), ("inv_tref", -1.0), ("search_chunk", -1), ("search_chunk", 65),
    ("search_blocks", -2), ("layout", 3), ("search_band", 63), ("search_band", -1),
    ("window_shape", 2), ("render_rays", 48), ("render_rays", 128), ("render_blocks", -1),
])
def test_invalid_params_rejected_on_host(field, value):
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    p = sc.params.replace(**{field: value})
    L = hp.lib()
    st = ctypes.c_int32()
    arr, pp = hp._cams_array(sc.cams), hp.make_params(p)
    n = L.hp_table_workspace(10, arr, 1, ctypes.byref(pp), ctypes.byref(st))
    if field == "K" and value == 33:
        # K is checked by the search (unsupported), not by the table
        return
    assert n == 0 and st.value == hp.HP_E_INVALID


def test_build_rejects_bad_arguments_without_launching():
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    L = hp.lib()
    arr, pp = hp._cams_array(sc.cams), hp.make_params(sc.params)
    tab = hp.HPTable()
    # null xyz with n > 0
    assert L.hp_build_table(None, 10, arr, 1, ctypes.byref(pp), None, 0, ctypes.byref(tab), None) == hp.HP_E_INVALID
    # no workspace
    fake = ctypes.c_void_p(0x1000)
    assert L.hp_build_table(fake, 10, arr, 1, ctypes.byref(pp), None, 0, ctypes.byref(tab), None) == hp.HP_E_WORKSPACE
    # too small a workspace
    assert L.hp_build_table(fake, 10, arr, 1, ctypes.byref(pp), fake, 16, ctypes.byref(tab), None) == hp.HP_E_WORKSPACE
    # too many views, bad camera
    assert L.hp_build_table(fake, 10, arr, 0, ctypes.byref(pp), fake, 1 << 30, ctypes.byref(tab), None) == hp.HP_E_INVALID
    bad = hp._cams_array(sc.cams)
    bad[0].fx = -1.0
    assert L.hp_build_table(fake, 10, bad, 1, ctypes.byref(pp), fake, 1 << 30, ctypes.byref(tab), None) == hp.HP_E_INVALID
    # n * views beyond int32 indices
    assert L.hp_build_table(fake, 1 << 31, arr, 1, ctypes.byref(pp), fake, 1 << 30, ctypes.byref(tab), None) == hp.HP_E_CAPACITY


def test_search_and_render_reject_bad_arguments_without_launching():
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    L = hp.lib()
    arr, pp = hp._cams_array(sc.cams), hp.make_params(sc.params)
    tab = hp.HPTable()  # all null pointers
    smp = hp.HPSamples()
    assert L.hp_search_sample(ctypes.byref(tab), arr, 1, ctypes.byref(pp), ctypes.byref(smp), None) == hp.HP_E_INVALID
    assert L.hp_search_sample(None, arr, 1, ctypes.byref(pp), ctypes.byref(smp), None) == hp.HP_E_INVALID
    mlp = hp.HPMlp()
    fake = ctypes.c_void_p(0x1000)
    # feature width other than 32
    assert L.hp_render(ctypes.byref(smp), 0, fake, 16, ctypes.byref(mlp), 0, ctypes.byref(pp), fake, None, None, None) == hp.HP_E_UNSUPPORTED
    # null weights
    assert L.hp_render(ctypes.byref(smp), 0, fake, 32, ctypes.byref(mlp), 0, ctypes.byref(pp), fake, None, None, None) == hp.HP_E_INVALID
    # bad precision
    assert L.hp_render(ctypes.byref(smp), 0, fake, 32, ctypes.byref(mlp), 7, ctypes.byref(pp), fake, None, None, None) == hp.HP_E_INVALID
    # backward with a null table
    assert L.hp_render_backward(None, arr, 1, fake, 32, ctypes.byref(mlp), 0, ctypes.byref(pp), fake, fake,
                                ctypes.byref(mlp), fake, 1 << 30, None) == hp.HP_E_INVALID


def test_backward_from_samples_rejects_bad_arguments_without_launching():
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    L = hp.lib()
    pp = hp.make_params(sc.params)
    fake = ctypes.c_void_p(0x1000)
    smp = hp.HPSamples()
    mlp = hp.HPMlp()
    for name, _ in hp.HPMlp._fields_:
        setattr(mlp, name, 0x1000)
    need = hp.backward_samples_workspace(sc.params)
    assert need > 0
    args = lambda s, R, C, prec, ws_bytes: (ctypes.byref(s) if s is not None else None, R, fake, C,
                                            ctypes.byref(mlp), prec, ctypes.byref(pp), fake, fake,
                                            ctypes.byref(mlp), fake, ws_bytes, None)
    # null sample arrays with rays to process
    assert L.hp_render_backward_samples(*args(smp, 10, 32, 0, need)) == hp.HP_E_INVALID
    assert L.hp_render_backward_samples(*args(None, 10, 32, 0, need)) == hp.HP_E_INVALID
    for name, _ in hp.HPSamples._fields_:
        setattr(smp, name, 0x1000)
    assert L.hp_render_backward_samples(*args(smp, 10, 16, 0, need)) == hp.HP_E_UNSUPPORTED
    assert L.hp_render_backward_samples(*args(smp, 10, 32, 5, need)) == hp.HP_E_INVALID
    assert L.hp_render_backward_samples(*args(smp, 10, 32, 0, need - 1)) == hp.HP_E_WORKSPACE
    assert L.hp_render_backward_samples(*args(smp, 1 << 31, 32, 0, need)) == hp.HP_E_CAPACITY
    assert L.hp_render_backward_samples(*args(smp, -1, 32, 0, need)) == hp.HP_E_INVALID


def test_backward_workspace_holds_one_chunk_of_recomputed_samples():
    """The recomputing backward's workspace holds the gradient slices and the
    samples of min(R, 262144) rays: it stops growing with the rays."""
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    part = hp.backward_samples_workspace(sc.params)
    st = ctypes.c_int32()
    tab = hp.HPTable()
    p = sc.params
    S, K = p.n_samples, p.K
    sizes = {}
    for R in (0, 1, 4096, 262144, 640000, 10_000_000):
        tab.n_rays = R
        n = hp.lib().hp_backward_workspace(ctypes.byref(tab), ctypes.byref(hp.make_params(p)),
                                           ctypes.byref(st))
        assert st.value == hp.HP_OK
        rays = max(1, min(R, 262144))
        assert n >= part + rays * (4 * 4 + S * 4 + 2 * S * K * 4)
        assert n <= part + rays * (4 * 4 + S * 4 + 2 * S * K * 4) + 8 * 256
        sizes[R] = n
    assert sizes[262144] == sizes[640000] == sizes[10_000_000]


def test_radius_modes_validated_and_bounded_like_the_oracle():
    import oracle
    sc = scenes.objects_1m(n=1000, res=64)
    cam = sc.cams[0]
    for mode in (1, 2, 3):
        p = sc.params.replace(radius_mode=mode, rddot=scenes.eq3_rddot(mode, sc.params.radius,
                                                                       sc.params.t_near))
        g, _ = hp.view_bounds(cam, p)
        assert g == oracle.guard(cam, p)
        assert hp.paper_kernel_size(cam, p) == oracle.paper_s(cam, p)
    assert hp.paper_kernel_size(cam, sc.params) == oracle.paper_s(cam, sc.params)
    pp = hp.make_params(sc.params.replace(radius_mode=1, rddot=0.0))
    c = hp.make_camera(cam)
    g = ctypes.c_int32()
    assert hp.lib().hp_view_bounds(ctypes.byref(c), ctypes.byref(pp), ctypes.byref(g), None) == hp.HP_E_INVALID
    for mode, rdd in ((4, 0.01), (-1, 0.01), (0, 0.01), (2, 1.5), (3, float("nan"))):
        pp = hp.make_params(sc.params.replace(radius_mode=mode, rddot=rdd))
        assert hp.lib().hp_view_bounds(ctypes.byref(c), ctypes.byref(pp), ctypes.byref(g), None) == hp.HP_E_INVALID


def test_sampler_parameters_validated():
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    c = hp.make_camera(sc.cams[0])
    g = ctypes.c_int32()
    ok = [(0, 0), (1, 1), (1, 4096), (1, 1 << 24)]
    bad = [(0, 5), (1, 0), (1, -3), (1, (1 << 24) + 1), (2, 10), (-1, 0)]
    for sampler, steps in ok + bad:
        pp = hp.make_params(sc.params.replace(sampler=sampler, ms_steps=steps))
        st = hp.lib().hp_view_bounds(ctypes.byref(c), ctypes.byref(pp), ctypes.byref(g), None)
        assert st == (hp.HP_OK if (sampler, steps) in ok else hp.HP_E_INVALID), (sampler, steps)


def test_knp_blend_rejects_bad_arguments_without_launching():
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    L = hp.lib()
    arr, pp = hp._cams_array(sc.cams), hp.make_params(sc.params)
    fake = ctypes.c_void_p(0x1000)
    tab = hp.HPTable()
    assert L.hp_knp_blend(ctypes.byref(tab), arr, 1, ctypes.byref(pp), 8, fake, fake, None, None, None,
                          None) == hp.HP_E_INVALID
    assert L.hp_knp_blend(None, arr, 1, ctypes.byref(pp), 8, fake, fake, None, None, None,
                          None) == hp.HP_E_INVALID


def test_samples_shape_counts():
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    p = sc.params.replace(K=5, n_samples=7, m_cap=33)
    sh = hp.samples_shape(1000, p)
    assert (sh.n_rays, sh.sample_rows, sh.knn_entries, sh.nbr_entries) == (1000, 7000, 35000, 33000)
    assert hp.samples_shape(0, p).knn_entries == 0
    L = hp.lib()
    out = hp.HPShape()
    pp = hp.make_params(p)
    assert L.hp_samples_shape(-1, ctypes.byref(pp), ctypes.byref(out)) == hp.HP_E_INVALID
    assert L.hp_samples_shape(1 << 60, ctypes.byref(pp), ctypes.byref(out)) == hp.HP_E_CAPACITY
    bad = hp.make_params(p.replace(K=0))
    assert L.hp_samples_shape(10, ctypes.byref(bad), ctypes.byref(out)) == hp.HP_E_INVALID


def test_exp32_eval_rejects_bad_arguments():
    L = hp.lib()
    assert L.hp_exp32_eval(None, None, -1, None) == hp.HP_E_INVALID
    assert L.hp_exp32_eval(None, None, 4, None) == hp.HP_E_INVALID
    assert L.hp_exp32_eval(None, None, 0, None) == hp.HP_OK


def _fake_table(cam, params):
    """A table struct whose geometry matches (cam, params) but whose build key
    is not the one hp_build_table would have written."""
    g, d = hp.view_bounds(cam, params)
    tab = hp.HPTable()
    tab.n_views, tab.layout, tab.n_points = 1, int(params.layout), 100
    tab.n_buckets = (cam.W + 2 * g) * (cam.H + 2 * g)
    tab.n_rays = cam.W * cam.H
    for name in ("offsets", "pts", "perm", "pcam", "bucket_z", "cell_zmin", "scratch"):
        setattr(tab, name, 0x1000)
    v = tab.views[0]
    v.W, v.H, v.g, v.Wg, v.Hg = cam.W, cam.H, g, cam.W + 2 * g, cam.H + 2 * g
    tab.build_key = 12345
    return tab


def test_calls_on_a_table_check_its_build_key():
    """A table records a hash of the cameras and of the parameters its bounds
    depend on; a search with other values is rejected before any launch."""
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    L = hp.lib()
    arr, pp = hp._cams_array(sc.cams), hp.make_params(sc.params)
    tab = _fake_table(sc.cams[0], sc.params)
    smp = hp.HPSamples()
    for name, _ in hp.HPSamples._fields_[:7]:
        setattr(smp, name, 0x1000)
    assert L.hp_search_sample(ctypes.byref(tab), arr, 1, ctypes.byref(pp), ctypes.byref(smp),
                              None) == hp.HP_E_INVALID
    fake = ctypes.c_void_p(0x1000)
    assert L.hp_knp_blend(ctypes.byref(tab), arr, 1, ctypes.byref(pp), 8, fake, fake, None, None,
                          None, None) == hp.HP_E_INVALID
    mlp = hp.HPMlp()
    for name, _ in hp.HPMlp._fields_:
        setattr(mlp, name, 0x1000)
    assert L.hp_render_backward_noalloc(ctypes.byref(tab), arr, 1, fake, 32, ctypes.byref(mlp), 0,
                                        ctypes.byref(pp), fake, fake, ctypes.byref(mlp),
                                        None) == hp.HP_E_INVALID


def test_backward_noalloc_rejects_bad_arguments_without_launching():
    """The allocation-free backward validates like hp_render_backward (no
    workspace to check) before it touches a device or its scratch array."""
    sc = scenes.sphere_plane(n_sphere=10, n_plane=10)
    L = hp.lib()
    arr, pp = hp._cams_array(sc.cams), hp.make_params(sc.params)
    fake = ctypes.c_void_p(0x1000)
    mlp = hp.HPMlp()
    for name, _ in hp.HPMlp._fields_:
        setattr(mlp, name, 0x1000)
    f = L.hp_render_backward_noalloc
    args = lambda tab, C, prec, m: (tab, arr, 1, fake, C, m, prec, ctypes.byref(pp), fake, fake,
                                    m, None)
    tab = _fake_table(sc.cams[0], sc.params)
    assert f(*args(None, 32, 0, ctypes.byref(mlp))) == hp.HP_E_INVALID
    assert f(*args(ctypes.byref(tab), 32, 0, None)) == hp.HP_E_INVALID
    # a table whose build key does not match is rejected before the others
    assert f(*args(ctypes.byref(tab), 16, 0, ctypes.byref(mlp))) == hp.HP_E_INVALID
    bad = hp.make_params(sc.params)
    bad.K = 0
    assert f(ctypes.byref(tab), arr, 1, fake, 32, ctypes.byref(mlp), 0, ctypes.byref(bad), fake,
             fake, ctypes.byref(mlp), None) == hp.HP_E_INVALID
