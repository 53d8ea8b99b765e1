"""Python binding of libhashpoint.so (the C ABI in include/hashpoint.h).

Argument marshalling only: every step of the method runs in the library's HIP
kernels.  PyTorch supplies device memory and the current HIP stream.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhashpoint.so")

HP_OK, HP_E_INVALID, HP_E_WORKSPACE, HP_E_UNSUPPORTED, HP_E_CAPACITY, HP_E_HIP = range(6)
HP_FP32, HP_BF16 = 0, 1
HP_LAYOUT_ROWMAJOR, HP_LAYOUT_TILED, HP_LAYOUT_MORTON = 0, 1, 2
HP_WINDOW_DISC, HP_WINDOW_SQUARE = 0, 1
HP_RADIUS_LINEAR, HP_RADIUS_EQ3, HP_RADIUS_EQ3_AF, HP_RADIUS_EQ3_AE = 0, 1, 2, 3
HP_SAMPLER_PS, HP_SAMPLER_MS = 0, 1
HP_MAX_VIEWS = 32
FEAT_DIM = 32
HIDDEN = 64

EXPORTED = ["hp_table_workspace", "hp_view_bounds", "hp_paper_kernel_size", "hp_build_table", "hp_search_sample",
            "hp_render", "hp_backward_workspace", "hp_render_backward",
            "hp_backward_samples_workspace", "hp_render_backward_samples", "hp_knp_blend",
            "hp_search_render", "hp_samples_shape", "hp_exp32_eval",
            "hp_render_backward_noalloc", "hp_bf16_eval",
            "hp_status_str",
            "hp_last_hip_error"]


class HashPointError(RuntimeError):
    pass


class HPCamera(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("H", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("C", ctypes.c_float * 3)]


class HPParams(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_float), ("inv_tref", ctypes.c_float),
                ("t_near", ctypes.c_float), ("t_far", ctypes.c_float),
                ("K", ctypes.c_int32), ("n_samples", ctypes.c_int32), ("m_cap", ctypes.c_int32),
                ("gamma", ctypes.c_float), ("inv_beta2", ctypes.c_float),
                ("eps_w", ctypes.c_float), ("eps_idw", ctypes.c_float),
                ("delta_last", ctypes.c_float), ("bg", ctypes.c_float * 3),
                ("layout", ctypes.c_int32), ("flags", ctypes.c_int32),
                ("search_chunk", ctypes.c_int32), ("search_blocks", ctypes.c_int32),
                ("radius_mode", ctypes.c_int32), ("rddot", ctypes.c_float),
                ("sampler", ctypes.c_int32), ("ms_steps", ctypes.c_int32),
                ("search_band", ctypes.c_int32), ("window_shape", ctypes.c_int32),
                ("render_rays", ctypes.c_int32), ("render_blocks", ctypes.c_int32)]


class HPViewInfo(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("H", ctypes.c_int32), ("g", ctypes.c_int32),
                ("Wg", ctypes.c_int32), ("Hg", ctypes.c_int32),
                ("bucket_base", ctypes.c_int32), ("ray_base", ctypes.c_int32),
                ("delta_max", ctypes.c_float)]


class HPTable(ctypes.Structure):
    _fields_ = [("n_views", ctypes.c_int32), ("layout", ctypes.c_int32),
                ("n_points", ctypes.c_int64), ("n_buckets", ctypes.c_int64),
                ("n_rays", ctypes.c_int64),
                ("offsets", ctypes.c_void_p), ("pts", ctypes.c_void_p),
                ("perm", ctypes.c_void_p), ("pcam", ctypes.c_void_p),
                ("bucket_z", ctypes.c_void_p), ("cell_zmin", ctypes.c_void_p),
                ("n_cells", ctypes.c_int64), ("build_key", ctypes.c_uint64),
                ("scratch", ctypes.c_void_p), ("views", HPViewInfo * HP_MAX_VIEWS)]


class HPSamples(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in
                ("n_sel", "primary", "n_nbr", "flags", "t", "knn_idx", "knn_dist",
                 "nbr_idx", "nbr_t")]


class HPShape(ctypes.Structure):
    _fields_ = [(name, ctypes.c_int64) for name in
                ("n_rays", "sample_rows", "knn_entries", "nbr_entries")]


class HPMlp(ctypes.Structure):
    _fields_ = [(name, ctypes.c_void_p) for name in ("W1", "b1", "W2", "b2", "W3", "b3")]


_lib = None


def lib():
    """Load libhashpoint.so; raise if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise HashPointError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
        L.hp_table_workspace.restype = ctypes.c_size_t
        L.hp_table_workspace.argtypes = [i64, P, i32, P, P]
        L.hp_view_bounds.restype = i32
        L.hp_view_bounds.argtypes = [P, P, P, P]
        L.hp_paper_kernel_size.restype = i32
        L.hp_paper_kernel_size.argtypes = [P, P, P]
        L.hp_build_table.restype = i32
        L.hp_build_table.argtypes = [P, i64, P, i32, P, P, ctypes.c_size_t, P, P]
        L.hp_search_sample.restype = i32
        L.hp_search_sample.argtypes = [P, P, i32, P, P, P]
        L.hp_render.restype = i32
        L.hp_render.argtypes = [P, i64, P, i32, P, i32, P, P, P, P, P]
        L.hp_backward_workspace.restype = ctypes.c_size_t
        L.hp_backward_workspace.argtypes = [P, P, P]
        L.hp_render_backward.restype = i32
        L.hp_render_backward.argtypes = [P, P, i32, P, i32, P, i32, P, P, P, P, P, ctypes.c_size_t, P]
        L.hp_search_render.restype = i32
        L.hp_search_render.argtypes = [P, P, i32, P, P, i32, P, i32, P, P, P, P, P]
        L.hp_knp_blend.restype = i32
        L.hp_knp_blend.argtypes = [P, P, i32, P, i32, P, P, P, P, P, P]
        L.hp_backward_samples_workspace.restype = ctypes.c_size_t
        L.hp_backward_samples_workspace.argtypes = [P, P]
        L.hp_render_backward_samples.restype = i32
        L.hp_render_backward_samples.argtypes = [P, i64, P, i32, P, i32, P, P, P, P, P, ctypes.c_size_t, P]
        L.hp_render_backward_noalloc.restype = i32
        L.hp_render_backward_noalloc.argtypes = [P, P, i32, P, i32, P, i32, P, P, P, P, P]
        L.hp_samples_shape.restype = i32
        L.hp_samples_shape.argtypes = [i64, P, P]
        L.hp_exp32_eval.restype = i32
        L.hp_exp32_eval.argtypes = [P, P, i64, P]
        L.hp_bf16_eval.restype = i32
        L.hp_bf16_eval.argtypes = [P, P, i64, P]
        L.hp_status_str.restype = ctypes.c_char_p
        L.hp_status_str.argtypes = [i32]
        L.hp_last_hip_error.restype = i32
        L.hp_last_hip_error.argtypes = []
        _lib = L
    return _lib


def _check(status: int, what: str):
    if status != HP_OK:
        msg = lib().hp_status_str(status).decode()
        extra = f" (hip error {lib().hp_last_hip_error()})" if status == HP_E_HIP else ""
        raise HashPointError(f"{what}: {msg}{extra}")


def make_camera(cam) -> HPCamera:
    c = HPCamera()
    c.W, c.H = int(cam.W), int(cam.H)
    c.fx, c.fy, c.cx, c.cy = float(cam.fx), float(cam.fy), float(cam.cx), float(cam.cy)
    for i, v in enumerate(np.asarray(cam.R, np.float32).reshape(-1)):
        c.R[i] = float(v)
    for i, v in enumerate(np.asarray(cam.C, np.float32).reshape(-1)):
        c.C[i] = float(v)
    return c


def make_params(p) -> HPParams:
    s = HPParams()
    s.radius, s.inv_tref, s.t_near, s.t_far = p.radius, p.inv_tref, p.t_near, p.t_far
    s.K, s.n_samples, s.m_cap = int(p.K), int(p.n_samples), int(p.m_cap)
    s.gamma, s.inv_beta2, s.eps_w, s.eps_idw = p.gamma, p.inv_beta2, p.eps_w, p.eps_idw
    s.delta_last = p.delta_last
    for i in range(3):
        s.bg[i] = float(p.bg[i])
    s.layout, s.flags = int(getattr(p, "layout", 0)), int(getattr(p, "flags", 0))
    s.search_chunk = int(getattr(p, "search_chunk", 0))
    s.search_blocks = int(getattr(p, "search_blocks", 0))
    s.radius_mode = int(getattr(p, "radius_mode", 0))
    s.rddot = float(getattr(p, "rddot", 0.0))
    s.sampler = int(getattr(p, "sampler", 0))
    s.ms_steps = int(getattr(p, "ms_steps", 0))
    s.search_band = int(getattr(p, "search_band", 0))
    s.window_shape = int(getattr(p, "window_shape", 0))
    s.render_rays = int(getattr(p, "render_rays", 0))
    s.render_blocks = int(getattr(p, "render_blocks", 0))
    return s


def _cams_array(cams: Sequence) -> ctypes.Array:
    arr = (HPCamera * len(cams))()
    for i, c in enumerate(cams):
        arr[i] = c if isinstance(c, HPCamera) else make_camera(c)
    return arr


def _stream(stream=None) -> int:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev(t: torch.Tensor, dtype, name: str) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise HashPointError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise HashPointError(f"{name} must be a contiguous {dtype} tensor")
    return t.data_ptr()


def view_bounds(cam, params):
    g = ctypes.c_int32()
    d = ctypes.c_float()
    c, p = make_camera(cam), make_params(params)
    _check(lib().hp_view_bounds(ctypes.byref(c), ctypes.byref(p), ctypes.byref(g), ctypes.byref(d)),
           "hp_view_bounds")
    return g.value, d.value


def paper_kernel_size(cam, params) -> int:
    """The paper's search-kernel size s = 2 ceil(rddot / rdot) + 1 (Sec. 3.2)."""
    out = ctypes.c_int32()
    c, p = make_camera(cam), make_params(params)
    _check(lib().hp_paper_kernel_size(ctypes.byref(c), ctypes.byref(p), ctypes.byref(out)),
           "hp_paper_kernel_size")
    return out.value


def table_workspace(n: int, cams, params) -> int:
    st = ctypes.c_int32()
    arr, p = _cams_array(cams), make_params(params)
    nbytes = lib().hp_table_workspace(int(n), arr, len(cams), ctypes.byref(p), ctypes.byref(st))
    _check(st.value, "hp_table_workspace")
    return int(nbytes)


class Table:
    """A built pixel table; owns its workspace tensor."""

    def __init__(self, ws, tab, cams, params, xyz):
        self.ws, self.tab, self.cams, self.params, self.xyz = ws, tab, cams, params, xyz
        self.n_rays = int(tab.n_rays)
        self.n_points = int(tab.n_points)
        self.n_buckets = int(tab.n_buckets)

    def view(self, i):
        return self.tab.views[i]

    def offsets(self) -> torch.Tensor:
        n = self.n_buckets + 1
        return _wrap(self.ws, self.tab.offsets, n, torch.int32)

    def perm(self, n_in: int) -> torch.Tensor:
        return _wrap(self.ws, self.tab.perm, n_in, torch.int32)

    def pts(self, n_in: int) -> torch.Tensor:
        return _wrap(self.ws, self.tab.pts, 4 * n_in, torch.float32).view(n_in, 4)

    def bucket_z(self) -> torch.Tensor:
        """Depth of each bucket's first point (+inf if empty)."""
        return _wrap(self.ws, self.tab.bucket_z, self.n_buckets, torch.float32)

    def cell_zmin(self) -> torch.Tensor:
        """Minimum depth of each 8x8-bucket cell as binary32 bits (int32 view)."""
        return _wrap(self.ws, self.tab.cell_zmin, int(self.tab.n_cells), torch.int32)


def _wrap(ws: torch.Tensor, ptr: int, count: int, dtype) -> torch.Tensor:
    """View of `count` elements of workspace `ws` starting at device address ptr."""
    off = ptr - ws.data_ptr()
    itemsize = torch.empty((), dtype=dtype).element_size()
    assert off % itemsize == 0 and off >= 0 and off + count * itemsize <= ws.numel()
    return ws[off: off + count * itemsize].view(dtype)


def build_table(xyz: torch.Tensor, cams, params, ws: Optional[torch.Tensor] = None,
                stream=None) -> Table:
    n = int(xyz.shape[0])
    xp = _dev(xyz, torch.float32, "xyz")
    need = table_workspace(n, cams, params)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=xyz.device)
    arr, p = _cams_array(cams), make_params(params)
    tab = HPTable()
    _check(lib().hp_build_table(xp, n, arr, len(cams), ctypes.byref(p), ws.data_ptr(), ws.numel(),
                                ctypes.byref(tab), _stream(stream)), "hp_build_table")
    return Table(ws, tab, list(cams), params, xyz)


def samples_shape(n_rays: int, params) -> HPShape:
    """Element counts of the sample arrays for n_rays rays (hp_samples_shape)."""
    sh = HPShape()
    p = make_params(params)
    _check(lib().hp_samples_shape(int(n_rays), ctypes.byref(p), ctypes.byref(sh)), "hp_samples_shape")
    return sh


def alloc_samples(n_rays: int, params, device, debug: bool = False) -> Dict[str, torch.Tensor]:
    sh = samples_shape(n_rays, params)
    R = sh.n_rays
    out = {
        "n_sel": torch.empty(R, dtype=torch.int32, device=device),
        "primary": torch.empty(R, dtype=torch.int32, device=device),
        "n_nbr": torch.empty(R, dtype=torch.int32, device=device),
        "flags": torch.empty(R, dtype=torch.int32, device=device),
        "t": torch.empty(sh.sample_rows, dtype=torch.float32, device=device),
        "knn_idx": torch.empty(sh.knn_entries, dtype=torch.int32, device=device),
        "knn_dist": torch.empty(sh.knn_entries, dtype=torch.float32, device=device),
    }
    if debug:
        out["nbr_idx"] = torch.empty(sh.nbr_entries, dtype=torch.int32, device=device)
        out["nbr_t"] = torch.empty(sh.nbr_entries, dtype=torch.float32, device=device)
    return out


def exp32_eval(x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The device's binary32 exp of the candidate confidences, element-wise."""
    if out is None:
        out = torch.empty_like(x)
    _check(lib().hp_exp32_eval(_dev(x, torch.float32, "x"), _dev(out, torch.float32, "out"),
                               int(x.numel()), _stream(stream)), "hp_exp32_eval")
    return out


def bf16_eval(x: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """The device's rounding of binary32 values to bfloat16 (as binary32), element-wise."""
    if out is None:
        out = torch.empty_like(x)
    _check(lib().hp_bf16_eval(_dev(x, torch.float32, "x"), _dev(out, torch.float32, "out"),
                               int(x.numel()), _stream(stream)), "hp_bf16_eval")
    return out


def _samples_struct(s: Dict[str, torch.Tensor]) -> HPSamples:
    st = HPSamples()
    for name, _ in HPSamples._fields_:
        setattr(st, name, s[name].data_ptr() if name in s else None)
    return st


def search_sample(table: Table, params=None, out: Optional[Dict[str, torch.Tensor]] = None,
                  debug: bool = False, stream=None) -> Dict[str, torch.Tensor]:
    params = params or table.params
    if out is None:
        out = alloc_samples(table.n_rays, params, table.ws.device, debug)
    arr, p = _cams_array(table.cams), make_params(params)
    st = _samples_struct(out)
    _check(lib().hp_search_sample(ctypes.byref(table.tab), arr, len(table.cams), ctypes.byref(p),
                                  ctypes.byref(st), _stream(stream)), "hp_search_sample")
    return out


def mlp_struct(mlp: Dict[str, torch.Tensor]) -> HPMlp:
    m = HPMlp()
    for name in ("W1", "b1", "W2", "b2", "W3", "b3"):
        setattr(m, name, _dev(mlp[name], torch.float32, name))
    return m


def render(samples: Dict[str, torch.Tensor], n_rays: int, feat: torch.Tensor,
           mlp: Dict[str, torch.Tensor], params, precision: int = HP_FP32,
           out: Optional[Dict[str, torch.Tensor]] = None, stream=None) -> Dict[str, torch.Tensor]:
    dev = feat.device
    if out is None:
        out = {"rgb": torch.empty(n_rays * 3, dtype=torch.float32, device=dev),
               "depth": torch.empty(n_rays, dtype=torch.float32, device=dev),
               "acc": torch.empty(n_rays, dtype=torch.float32, device=dev)}
    fp = _dev(feat, torch.float32, "feat")
    st = _samples_struct(samples)
    m = mlp_struct(mlp)
    p = make_params(params)
    _check(lib().hp_render(ctypes.byref(st), int(n_rays), fp, int(feat.shape[1]), ctypes.byref(m),
                           int(precision), ctypes.byref(p), out["rgb"].data_ptr(),
                           out["depth"].data_ptr() if out.get("depth") is not None else None,
                           out["acc"].data_ptr() if out.get("acc") is not None else None,
                           _stream(stream)), "hp_render")
    return out


def search_render(table: Table, params, feat: torch.Tensor, mlp: Dict[str, torch.Tensor],
                  precision: int, out: Optional[Dict[str, torch.Tensor]] = None,
                  stream=None) -> Dict[str, torch.Tensor]:
    """search_sample + render in one launch (samples stay on chip)."""
    params = params or table.params
    R, dev = table.n_rays, feat.device
    if out is None:
        out = {"rgb": torch.empty(R * 3, device=dev), "depth": torch.empty(R, device=dev),
               "acc": torch.empty(R, device=dev), "n_sel": torch.empty(R, dtype=torch.int32, device=dev)}
    arr, p, m = _cams_array(table.cams), make_params(params), mlp_struct(mlp)
    _check(lib().hp_search_render(ctypes.byref(table.tab), arr, len(table.cams), ctypes.byref(p),
                                  _dev(feat, torch.float32, "feat"), int(feat.shape[1]),
                                  ctypes.byref(m), int(precision), out["rgb"].data_ptr(),
                                  out["depth"].data_ptr() if out.get("depth") is not None else None,
                                  out["acc"].data_ptr() if out.get("acc") is not None else None,
                                  out["n_sel"].data_ptr() if out.get("n_sel") is not None else None,
                                  _stream(stream)), "hp_search_render")
    return out


def knp_blend(table: Table, params, K: int, colors: torch.Tensor, lists: bool = True,
              out: Optional[Dict[str, torch.Tensor]] = None, stream=None) -> Dict[str, torch.Tensor]:
    """K nearest points to every ray and their Eq. 1 blend of per-point colours."""
    params = params or table.params
    R, dev = table.n_rays, table.ws.device
    if out is None:
        out = {"rgb": torch.empty(R * 3, dtype=torch.float32, device=dev),
               "cnt": torch.empty(R, dtype=torch.int32, device=dev)}
        if lists:
            out["idx"] = torch.empty(R * K, dtype=torch.int32, device=dev)
            out["dist"] = torch.empty(R * K, dtype=torch.float32, device=dev)
    arr, p = _cams_array(table.cams), make_params(params)
    _check(lib().hp_knp_blend(ctypes.byref(table.tab), arr, len(table.cams), ctypes.byref(p), int(K),
                              _dev(colors, torch.float32, "colors"), out["rgb"].data_ptr(),
                              out["cnt"].data_ptr() if "cnt" in out else None,
                              out["idx"].data_ptr() if "idx" in out else None,
                              out["dist"].data_ptr() if "dist" in out else None, _stream(stream)),
           "hp_knp_blend")
    return out


def to_device_mlp(mlp: Dict[str, np.ndarray], device) -> Dict[str, torch.Tensor]:
    return {k: torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(device) for k, v in mlp.items()}


def backward_workspace(table: Table, params=None) -> int:
    st = ctypes.c_int32()
    p = make_params(params or table.params)
    n = lib().hp_backward_workspace(ctypes.byref(table.tab), ctypes.byref(p), ctypes.byref(st))
    _check(st.value, "hp_backward_workspace")
    return int(n)


def render_backward(table: Table, feat: torch.Tensor, mlp: Dict[str, torch.Tensor], params,
                    precision: int, grad_rgb: torch.Tensor,
                    grad_feat: Optional[torch.Tensor] = None,
                    grad_mlp: Optional[Dict[str, torch.Tensor]] = None,
                    ws: Optional[torch.Tensor] = None, stream=None):
    """Gradients of sum(grad_rgb * rgb) w.r.t. features and MLP parameters.
    Results are added to grad_feat / grad_mlp (zero-initialised when not given)."""
    params = params or table.params
    dev = feat.device
    if grad_feat is None:
        grad_feat = torch.zeros_like(feat)
    if grad_mlp is None:
        grad_mlp = {k: torch.zeros_like(v) for k, v in mlp.items()}
    if ws is None:
        # (a caller's workspace is used as given: any size that holds one ray's
        # samples works, a smaller one just means more recompute chunks)
        ws = torch.empty(backward_workspace(table, params), dtype=torch.uint8, device=dev)
    arr, p = _cams_array(table.cams), make_params(params)
    m, gm = mlp_struct(mlp), mlp_struct(grad_mlp)
    _check(lib().hp_render_backward(ctypes.byref(table.tab), arr, len(table.cams),
                                    _dev(feat, torch.float32, "feat"), int(feat.shape[1]),
                                    ctypes.byref(m), int(precision), ctypes.byref(p),
                                    _dev(grad_rgb, torch.float32, "grad_rgb"),
                                    _dev(grad_feat, torch.float32, "grad_feat"), ctypes.byref(gm),
                                    ws.data_ptr(), ws.numel(), _stream(stream)),
           "hp_render_backward")
    return grad_feat, grad_mlp


def render_backward_noalloc(table: Table, feat: torch.Tensor, mlp: Dict[str, torch.Tensor], params,
                            precision: int, grad_rgb: torch.Tensor,
                            grad_feat: torch.Tensor, grad_mlp: Dict[str, torch.Tensor], stream=None):
    """render_backward without a workspace: the library's per-GPU scratch array
    holds the gradient slices and the recompute ring, and the call allocates
    nothing (grad_feat / grad_mlp are given by the caller and added to)."""
    params = params or table.params
    arr, p = _cams_array(table.cams), make_params(params)
    m, gm = mlp_struct(mlp), mlp_struct(grad_mlp)
    _check(lib().hp_render_backward_noalloc(ctypes.byref(table.tab), arr, len(table.cams),
                                            _dev(feat, torch.float32, "feat"), int(feat.shape[1]),
                                            ctypes.byref(m), int(precision), ctypes.byref(p),
                                            _dev(grad_rgb, torch.float32, "grad_rgb"),
                                            _dev(grad_feat, torch.float32, "grad_feat"),
                                            ctypes.byref(gm), _stream(stream)),
           "hp_render_backward_noalloc")
    return grad_feat, grad_mlp


def backward_samples_workspace(params) -> int:
    st = ctypes.c_int32()
    p = make_params(params)
    n = lib().hp_backward_samples_workspace(ctypes.byref(p), ctypes.byref(st))
    _check(st.value, "hp_backward_samples_workspace")
    return int(n)


def render_backward_samples(samples: Dict[str, torch.Tensor], n_rays: int, feat: torch.Tensor,
                            mlp: Dict[str, torch.Tensor], params, precision: int,
                            grad_rgb: torch.Tensor, grad_feat: Optional[torch.Tensor] = None,
                            grad_mlp: Optional[Dict[str, torch.Tensor]] = None,
                            ws: Optional[torch.Tensor] = None, stream=None):
    """render_backward from kept samples (as written by search_sample)."""
    dev = feat.device
    if grad_feat is None:
        grad_feat = torch.zeros_like(feat)
    if grad_mlp is None:
        grad_mlp = {k: torch.zeros_like(v) for k, v in mlp.items()}
    need = backward_samples_workspace(params)
    if ws is None or ws.numel() < need:
        ws = torch.empty(need, dtype=torch.uint8, device=dev)
    st, p = _samples_struct(samples), make_params(params)
    m, gm = mlp_struct(mlp), mlp_struct(grad_mlp)
    _check(lib().hp_render_backward_samples(ctypes.byref(st), int(n_rays),
                                            _dev(feat, torch.float32, "feat"), int(feat.shape[1]),
                                            ctypes.byref(m), int(precision), ctypes.byref(p),
                                            _dev(grad_rgb, torch.float32, "grad_rgb"),
                                            _dev(grad_feat, torch.float32, "grad_feat"),
                                            ctypes.byref(gm), ws.data_ptr(), ws.numel(),
                                            _stream(stream)),
           "hp_render_backward_samples")
    return grad_feat, grad_mlp


_MLP_KEYS = ("W1", "b1", "W2", "b2", "W3", "b3")


class HashPointRender(torch.autograd.Function):
    """rgb = render(search_sample(table), feat, mlp) with a hand-written backward.

    By default the forward keeps no sample lists and the backward recomputes
    the search and sampling from the table (they depend on geometry only);
    with keep_samples=True the forward's samples are kept for the backward
    instead (more memory, no second search)."""

    @staticmethod
    def forward(ctx, feat, W1, b1, W2, b2, W3, b3, table, params, precision, keep_samples=False):
        mlp = dict(zip(_MLP_KEYS, (W1, b1, W2, b2, W3, b3)))
        smp = search_sample(table, params)
        out = render(smp, table.n_rays, feat, mlp, params, precision)
        ctx.samples = smp if keep_samples else None
        del smp
        ctx.table, ctx.params, ctx.precision = table, params, precision
        ctx.save_for_backward(feat, W1, b1, W2, b2, W3, b3)
        return out["rgb"].view(table.n_rays, 3)

    @staticmethod
    def backward(ctx, grad_rgb):
        feat, W1, b1, W2, b2, W3, b3 = ctx.saved_tensors
        mlp = dict(zip(_MLP_KEYS, (W1, b1, W2, b2, W3, b3)))
        g = grad_rgb.contiguous().float()
        if ctx.samples is not None:
            gf, gm = render_backward_samples(ctx.samples, ctx.table.n_rays, feat, mlp, ctx.params,
                                             ctx.precision, g)
            ctx.samples = None
        else:
            gf, gm = render_backward(ctx.table, feat, mlp, ctx.params, ctx.precision, g)
        return (gf, gm["W1"], gm["b1"], gm["W2"], gm["b2"], gm["W3"], gm["b3"], None, None, None,
                None)
