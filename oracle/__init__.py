"""CPU oracle for the HashPoint hot path (arXiv 2404.14044) -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never loads it.  It wraps the plain C
implementation in ``oracle.c`` (brute-force neighbour search, candidate walk,
binary64 render and gradient) through ctypes.

Parity status: every function is pinned by ``tests/test_oracle_*.py`` against
closed forms, special cases, invariants, brute force in binary64 and central
finite differences.  The paper prints no worked numeric example, so no value is
pinned to a number printed in the paper.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-mavx2", "-mfma", "-Wall", "-Wno-unknown-pragmas"]


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so next to it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class Camera(ctypes.Structure):
    _fields_ = [("W", ctypes.c_int32), ("H", ctypes.c_int32),
                ("fx", ctypes.c_float), ("fy", ctypes.c_float),
                ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("R", ctypes.c_float * 9), ("C", ctypes.c_float * 3)]


class Params(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_float), ("inv_tref", ctypes.c_float),
                ("t_near", ctypes.c_float), ("t_far", ctypes.c_float),
                ("K", ctypes.c_int32), ("n_samples", ctypes.c_int32), ("m_cap", ctypes.c_int32),
                ("gamma", ctypes.c_float), ("inv_beta2", ctypes.c_float),
                ("eps_w", ctypes.c_float), ("eps_idw", ctypes.c_float),
                ("delta_last", ctypes.c_float), ("bg", ctypes.c_float * 3),
                ("radius_mode", ctypes.c_int32), ("rddot", ctypes.c_float),
                ("sampler", ctypes.c_int32), ("ms_steps", ctypes.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        _lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        i64, i32 = ctypes.c_int64, ctypes.c_int32
        _lib.or_exp32.restype = ctypes.c_float
        _lib.or_exp32.argtypes = [ctypes.c_float]
        _lib.or_exp32_array.argtypes = [P, P, i64]
        _lib.or_bf16_array.argtypes = [P, P, i64]
        _lib.or_guard.restype = i32
        _lib.or_guard.argtypes = [P, P]
        _lib.or_to_camera.argtypes = [P, i64, P, P]
        _lib.or_table.restype = i64
        _lib.or_table.argtypes = [P, i64, P, i32, P, P]
        _lib.or_ray_dir.argtypes = [P, i32, i32, P]
        _lib.or_knp.argtypes = [P, i64, P, P, P, i64, i32, P, P, P, P, P]
        _lib.or_paper_s.restype = i32
        _lib.or_paper_s.argtypes = [P, P]
        _lib.or_kappa.restype = ctypes.c_float
        _lib.or_kappa.argtypes = [P, ctypes.c_float, ctypes.c_float, ctypes.c_float]
        _lib.or_ray_kappa.restype = ctypes.c_float
        _lib.or_ray_kappa.argtypes = [P, P, i32, i32]
        _lib.or_exact.argtypes = [P, i64, P, P, P, i64] + [P] * 14
        _lib.or_render64.argtypes = [P, P, i32] + [P] * 6 + [P, P, P, i64, P, P, P, P, P, P]
        _lib.or_grad64.argtypes = [P, P, i32] + [P] * 6 + [P, P, P, i64, P, P, P, P, P] + [P] * 6
        _lib.or_render64q.argtypes = ([P, P, i32] + [P] * 6 + [P, P, P, i64, P, P, P, i32, P, P]
                                      + [P, P, P])
        _lib.or_grad64q.argtypes = ([P, P, i32] + [P] * 6 + [P, P, P, i64, P, P, P, i32, P, P]
                                    + [P, P] + [P] * 6)
        _lib.or_bf16.restype = ctypes.c_double
        _lib.or_bf16.argtypes = [ctypes.c_double]
        _lib.or_num_threads.restype = i32
        _lib.or_set_num_threads.argtypes = [i32]
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def camera_struct(cam) -> Camera:
    c = Camera()
    c.W, c.H = int(cam.W), int(cam.H)
    c.fx, c.fy, c.cx, c.cy = cam.fx, cam.fy, cam.cx, cam.cy
    for i, v in enumerate(np.asarray(cam.R, np.float32).reshape(-1)):
        c.R[i] = float(v)
    for i, v in enumerate(np.asarray(cam.C, np.float32).reshape(-1)):
        c.C[i] = float(v)
    return c


def params_struct(p) -> Params:
    s = Params()
    s.radius, s.inv_tref, s.t_near, s.t_far = p.radius, p.inv_tref, p.t_near, p.t_far
    s.K, s.n_samples, s.m_cap = int(p.K), int(p.n_samples), int(p.m_cap)
    s.gamma, s.inv_beta2, s.eps_w, s.eps_idw = p.gamma, p.inv_beta2, p.eps_w, p.eps_idw
    s.delta_last = p.delta_last
    for i in range(3):
        s.bg[i] = float(p.bg[i])
    s.radius_mode = int(getattr(p, "radius_mode", 0))
    s.rddot = float(getattr(p, "rddot", 0.0))
    s.sampler = int(getattr(p, "sampler", 0))
    s.ms_steps = int(getattr(p, "ms_steps", 0))
    return s


def num_threads() -> int:
    return int(lib().or_num_threads())


def set_num_threads(n: int) -> None:
    """Threads the oracle's parallel loops use from now on."""
    lib().or_set_num_threads(int(n))


def exp32(x) -> np.ndarray:
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().or_exp32_array(_ptr(x), _ptr(y), x.size)
    return y


def bf16_f32(x) -> np.ndarray:
    """Binary32 values rounded to bfloat16 (or_bf16), as binary32."""
    x = np.ascontiguousarray(x, np.float32)
    y = np.empty_like(x)
    lib().or_bf16_array(_ptr(x), _ptr(y), x.size)
    return y


def guard(cam, params) -> int:
    c, p = camera_struct(cam), params_struct(params)
    return int(lib().or_guard(ctypes.byref(c), ctypes.byref(p)))


def paper_s(cam, params) -> int:
    """The paper's kernel size s = 2 ceil(rddot / rdot) + 1 (Sec. 3.2)."""
    c, p = camera_struct(cam), params_struct(params)
    return int(lib().or_paper_s(ctypes.byref(c), ctypes.byref(p)))


def kappa(params, a: float, b: float, L: float) -> float:
    """Cone slope of Eq. 3 (rho = kappa t) for normalised pixel coordinates."""
    p = params_struct(params)
    return float(lib().or_kappa(ctypes.byref(p), ctypes.c_float(a), ctypes.c_float(b),
                                ctypes.c_float(L)))


def ray_kappa(cam, params, u: int, v: int) -> float:
    c, p = camera_struct(cam), params_struct(params)
    return float(lib().or_ray_kappa(ctypes.byref(c), ctypes.byref(p), int(u), int(v)))


def to_camera(xyz: np.ndarray, cam) -> np.ndarray:
    xyz = np.ascontiguousarray(xyz, np.float32)
    pc = np.empty_like(xyz)
    c = camera_struct(cam)
    lib().or_to_camera(_ptr(xyz), xyz.shape[0], ctypes.byref(c), _ptr(pc))
    return pc


def table(pc: np.ndarray, cam, g: int):
    """Returns (key[n] int32 (-1 = not inserted), order[n_in] int32)."""
    pc = np.ascontiguousarray(pc, np.float32)
    n = pc.shape[0]
    key = np.empty(n, np.int32)
    order = np.empty(max(n, 1), np.int32)
    c = camera_struct(cam)
    n_in = lib().or_table(_ptr(pc), n, ctypes.byref(c), int(g), _ptr(key), _ptr(order))
    return key, order[:n_in].copy()


def ray_dir(cam, u: int, v: int) -> np.ndarray:
    d = np.empty(3, np.float32)
    c = camera_struct(cam)
    lib().or_ray_dir(ctypes.byref(c), int(u), int(v), _ptr(d))
    return d


def knp(pc: np.ndarray, cam, params, K: int, colors: np.ndarray,
        pix: Optional[Sequence[int]] = None) -> Dict[str, np.ndarray]:
    """K nearest points to each ray among its neighbours and their Eq. 1 blend."""
    pc = np.ascontiguousarray(pc, np.float32)
    colors = np.ascontiguousarray(colors, np.float32)
    if pix is None:
        pix = np.arange(cam.W * cam.H, dtype=np.int32)
    pix = np.ascontiguousarray(pix, np.int32)
    R = pix.size
    out = {"cnt": np.empty(R, np.int32), "idx": np.empty((R, K), np.int32),
           "dist": np.empty((R, K), np.float32), "rgb": np.empty((R, 3), np.float64)}
    c, p = camera_struct(cam), params_struct(params)
    lib().or_knp(_ptr(pc), pc.shape[0], ctypes.byref(c), ctypes.byref(p), _ptr(pix), R, int(K),
                 _ptr(colors), _ptr(out["cnt"]), _ptr(out["idx"]), _ptr(out["dist"]), _ptr(out["rgb"]))
    return out


def exact(pc: np.ndarray, cam, params, pix: Optional[Sequence[int]] = None,
          diagnostics: bool = False) -> Dict[str, np.ndarray]:
    """Exact stage (search + candidate walk) for pixel indices ``pix`` (default: all)."""
    pc = np.ascontiguousarray(pc, np.float32)
    if pix is None:
        pix = np.arange(cam.W * cam.H, dtype=np.int32)
    pix = np.ascontiguousarray(pix, np.int32)
    R = pix.size
    M, S, K = params.m_cap, params.n_samples, params.K
    out = {
        "n_nbr": np.empty(R, np.int32), "flags": np.empty(R, np.uint32),
        "nbr_idx": np.empty((R, M), np.int32), "nbr_t": np.empty((R, M), np.float32),
        "n_sel": np.empty(R, np.int32), "primary": np.empty(R, np.int32),
        "t": np.empty((R, S), np.float32), "knn_idx": np.empty((R, S, K), np.int32),
        "knn_dist": np.empty((R, S, K), np.float32), "knn_cnt": np.empty((R, S), np.int32),
    }
    diag = [None] * 4
    if diagnostics:
        for name in ("cand_d", "cand_alpha", "cand_w", "cand_T"):
            out[name] = np.empty((R, M), np.float32)
        diag = [out["cand_d"], out["cand_alpha"], out["cand_w"], out["cand_T"]]
    c, p = camera_struct(cam), params_struct(params)
    lib().or_exact(_ptr(pc), pc.shape[0], ctypes.byref(c), ctypes.byref(p), _ptr(pix), R,
                   _ptr(out["n_nbr"]), _ptr(out["flags"]), _ptr(out["nbr_idx"]), _ptr(out["nbr_t"]),
                   _ptr(out["n_sel"]), _ptr(out["primary"]), _ptr(out["t"]), _ptr(out["knn_idx"]),
                   _ptr(out["knn_dist"]), _ptr(out["knn_cnt"]), *[_ptr(a) for a in diag])
    out["pix"] = pix
    return out


def _mlp_ptrs(mlp):
    arrs = [np.ascontiguousarray(mlp[k], np.float32) for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
    return arrs, [_ptr(a) for a in arrs]


QUANT_NONE, QUANT_BF16, QUANT_FROZEN = 0, 1, 2
N_ACT_OFF = 32 + 2 * 64  # per-sample operand offsets: aggregated feature, h1, h2


class QuantOffsets:
    """Rounding offsets bf16(x) - x of the decoder operands, recorded by a
    QUANT_BF16 call and replayed (held fixed) by QUANT_FROZEN calls on the
    same rays: the weights' offsets and, per sample row, those of the
    aggregated feature and the two hidden activations."""

    def __init__(self, n_rays: int, params, C: int = 32):
        n_w = 64 * C + 64 * 64 + 4 * 64
        self.w = np.zeros(n_w, np.float64)
        self.act = np.zeros(max(n_rays * params.n_samples, 1) * (C + 128), np.float64)


def bf16(x):
    """Round binary64 values to bfloat16 (8 significant bits, ties to even)."""
    f = lib().or_bf16
    return np.vectorize(lambda v: f(float(v)), otypes=[np.float64])(np.asarray(x, np.float64))


def _quant_args(quant, offsets):
    if quant == QUANT_NONE:
        return [0, None, None]
    if offsets is None:
        if quant == QUANT_FROZEN:
            raise ValueError("QUANT_FROZEN replays recorded offsets: pass offsets")
        return [int(quant), None, None]
    return [int(quant), _ptr(offsets.w), _ptr(offsets.act)]


def render64(pc, feat, mlp, cam, params, ex, quant: int = QUANT_NONE,
             offsets: Optional[QuantOffsets] = None) -> Dict[str, np.ndarray]:
    """Binary64 render of the exact stage's samples ``ex`` (from :func:`exact`).
    quant: QUANT_NONE, QUANT_BF16 (decoder operands rounded to bfloat16;
    records their offsets into ``offsets`` when given) or QUANT_FROZEN (the
    recorded offsets held fixed)."""
    pc = np.ascontiguousarray(pc, np.float32)
    feat = np.ascontiguousarray(feat, np.float32)
    keep, mp = _mlp_ptrs(mlp)
    R = ex["pix"].size
    rgb = np.empty((R, 3), np.float64)
    depth = np.empty(R, np.float64)
    acc = np.empty(R, np.float64)
    c, p = camera_struct(cam), params_struct(params)
    n_sel = np.ascontiguousarray(ex["n_sel"], np.int32)
    t = np.ascontiguousarray(ex["t"], np.float32)
    ki = np.ascontiguousarray(ex["knn_idx"], np.int32)
    lib().or_render64q(_ptr(pc), _ptr(feat), feat.shape[1], *mp, ctypes.byref(c), ctypes.byref(p),
                       _ptr(ex["pix"]), R, _ptr(n_sel), _ptr(t), _ptr(ki),
                       *_quant_args(quant, offsets), _ptr(rgb), _ptr(depth), _ptr(acc))
    return {"rgb": rgb, "depth": depth, "acc": acc}


def grad64(pc, feat, mlp, cam, params, ex, grad_rgb, quant: int = QUANT_NONE,
           offsets: Optional[QuantOffsets] = None) -> Dict[str, np.ndarray]:
    """Binary64 gradient of sum(grad_rgb * rgb) w.r.t. features and MLP
    parameters; quant as for :func:`render64` (roundings count as fixed
    offsets)."""
    pc = np.ascontiguousarray(pc, np.float32)
    feat = np.ascontiguousarray(feat, np.float32)
    keep, mp = _mlp_ptrs(mlp)
    R = ex["pix"].size
    g = np.ascontiguousarray(grad_rgb, np.float64).reshape(R, 3)
    out = {"feat": np.zeros(feat.shape, np.float64)}
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        out[k] = np.zeros(np.asarray(mlp[k]).shape, np.float64)
    c, p = camera_struct(cam), params_struct(params)
    n_sel = np.ascontiguousarray(ex["n_sel"], np.int32)
    t = np.ascontiguousarray(ex["t"], np.float32)
    ki = np.ascontiguousarray(ex["knn_idx"], np.int32)
    lib().or_grad64q(_ptr(pc), _ptr(feat), feat.shape[1], *mp, ctypes.byref(c), ctypes.byref(p),
                     _ptr(ex["pix"]), R, _ptr(n_sel), _ptr(t), _ptr(ki),
                     *_quant_args(quant, offsets), _ptr(g), _ptr(out["feat"]),
                     *[_ptr(out[k]) for k in ("W1", "b1", "W2", "b2", "W3", "b3")])
    return out
