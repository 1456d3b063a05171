"""Thin Python binding of libkk.so (ctypes).  Argument marshalling only: every step of
the method runs inside the library (host entry points in C++, device entry points as
gfx950 kernels).  Device buffers are torch tensors on the current HIP device; torch is
used for device memory and streams only.  The library must have been built (see
build.py); importing this module without it raises instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

try:  # torch first, so libkk binds to the HIP runtime torch has already loaded
    import torch
except ImportError:  # pragma: no cover - host-only use (selection, tables, plans)
    torch = None

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkk.so")

KK_OK, KK_E_NULL, KK_E_ARG, KK_E_CAPACITY, KK_E_WORKSPACE, KK_E_RANGE, KK_E_HIP, KK_E_UNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
SCHEME_SHIFTED, SCHEME_CONFOCAL, SCHEME_SAME, SCHEME_FULL_UNIFORM = 0, 1, 2, 3
PREC_FP32, PREC_BF16X3, PREC_FP16X3 = 0, 1, 2
COMPOUND_COHERENT, COMPOUND_INCOHERENT = 0, 1

EXPORTS = [
    "kk_select_pairs", "kk_build_luts", "kk_build_das_rx", "kk_beamform_plan",
    "kk_decompose_workspace_bytes", "kk_decompose", "kk_beamform_workspace_bytes", "kk_beamform",
    "kk_compound", "das_plan", "das_workspace_bytes", "das_beamform", "kk_status_string",
]


class KKError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__("%s failed: %s" % (fn, msg))
        self.status = status


class Geom(ctypes.Structure):
    _fields_ = [("L", ctypes.c_int32), ("T", ctypes.c_int32), ("pitch_m", ctypes.c_double),
                ("c_mps", ctypes.c_double), ("fs_hz", ctypes.c_double), ("t0_s", ctypes.c_double)]


class Grid(ctypes.Structure):
    _fields_ = [("X", ctypes.c_int32), ("Z", ctypes.c_int32), ("x0_m", ctypes.c_double),
                ("dx_m", ctypes.c_double), ("z0_m", ctypes.c_double), ("dz_m", ctypes.c_double)]


_lib = None
_i32p = ctypes.POINTER(ctypes.c_int32)
_dp = ctypes.POINTER(ctypes.c_double)
_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_szp = ctypes.POINTER(ctypes.c_size_t)
_i32 = ctypes.c_int32


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libkk.so is not built; run paper_2603_22496_amd.build.build_all()")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "kk_select_pairs": [_i32, _i32, _i32, ctypes.c_double, _i32, _i32p, _i32, _dp, _dp, _i32p, _i32p,
                                _i32, _i32p, _i32p, _i32, _i32p, _i32p, _dp],
            "kk_build_luts": [ctypes.POINTER(Geom), ctypes.POINTER(Grid), _dp, _i32, _dp, _i32, _i32p, _i32p,
                              _i32p, _i32p, _i32p, _i32p, _i32p],
            "kk_build_das_rx": [ctypes.POINTER(Geom), ctypes.POINTER(Grid), _i32p],
            "kk_beamform_plan": [_i32p, _i32, _i32, _i32, _i32, _i32, _i32p, _i32p, _i32p, _i32p, _i32,
                                 ctypes.POINTER(Grid), _vp, _sz, _szp],
            "kk_decompose": [_vp, _i32, ctypes.POINTER(Geom), _vp, _i32, _i32, _i32, _vp, _vp, _sz, _vp],
            "kk_beamform": [_vp, _i32, _i32, _i32, _vp, _vp, _sz, _vp, _vp, _i32, _vp, _sz, _vp],
            "kk_compound": [_vp, _i32, _i32, _i32, _i32, _vp, _vp],
            "das_plan": [_i32, ctypes.POINTER(Geom), _i32p, _i32p, _i32p, _i32, ctypes.POINTER(Grid), _vp, _sz,
                         _szp],
            "das_beamform": [_vp, _i32, ctypes.POINTER(Geom), _vp, _vp, _sz, _vp, _vp, _sz, _vp],
        }
        for name in EXPORTS:
            fn = getattr(L, name)
            if name in sig:
                fn.argtypes = sig[name]
                fn.restype = _i32
        L.kk_decompose_workspace_bytes.argtypes = [ctypes.POINTER(Geom), _i32, _i32, _i32, _i32]
        L.kk_decompose_workspace_bytes.restype = _sz
        L.das_workspace_bytes.argtypes = [ctypes.POINTER(Geom), _i32, _vp, _sz]
        L.das_workspace_bytes.restype = _sz
        L.kk_beamform_workspace_bytes.argtypes = [_vp, _sz]
        L.kk_beamform_workspace_bytes.restype = _sz
        L.kk_status_string.argtypes = [_i32]
        L.kk_status_string.restype = ctypes.c_char_p
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().kk_status_string(status).decode()


def _check(fn: str, status: int):
    if status != KK_OK:
        raise KKError(fn, status, status_string(status))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(_i32p)


def _dpp(a: np.ndarray):
    return a.ctypes.data_as(_dp)


def _dev(t) -> int:
    if torch is None or not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("device tensor must be contiguous")
    return t.data_ptr()


def _stream(stream) -> int:
    if stream is None:
        return torch.cuda.current_stream().cuda_stream
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)


def geom(L, T, pitch, c, fs, t0=0.0) -> Geom:
    return Geom(L, T, pitch, c, fs, t0)


def grid(X, Z, x0, dx, z0, dz) -> Grid:
    return Grid(X, Z, x0, dx, z0, dz)


# --------------------------------------------------------------------------- host calls

def select_pairs(scheme: int, L: int, N: int, theta_max: float, M: int, j_list=(0,)) -> dict:
    jl = np.ascontiguousarray(np.asarray(list(j_list), dtype=np.int32))
    tx = np.zeros(max(N, 1), dtype=np.float64)
    m_out, p_out, s_out = _i32(0), _i32(0), _i32(0)
    comp = ctypes.c_double(0.0)
    dummy_d = np.zeros(1)
    dummy_i = np.zeros(3, dtype=np.int32)
    st = lib().kk_select_pairs(scheme, L, N, theta_max, M, _ip(jl), len(jl), _dpp(tx), _dpp(dummy_d),
                               _ip(dummy_i), _ip(dummy_i), 0, ctypes.byref(m_out), _ip(dummy_i), 0,
                               ctypes.byref(p_out), ctypes.byref(s_out), ctypes.byref(comp))
    if st != KK_E_CAPACITY:
        _check("kk_select_pairs", st)
    Md, P = m_out.value, p_out.value
    rx = np.zeros(Md, dtype=np.float64)
    num = np.zeros(Md, dtype=np.int32)
    den = np.zeros(Md, dtype=np.int32)
    pairs = np.zeros((P, 3), dtype=np.int32)
    st = lib().kk_select_pairs(scheme, L, N, theta_max, M, _ip(jl), len(jl), _dpp(tx), _dpp(rx), _ip(num),
                               _ip(den), Md, ctypes.byref(m_out), _ip(pairs), P, ctypes.byref(p_out),
                               ctypes.byref(s_out), ctypes.byref(comp))
    _check("kk_select_pairs", st)
    return dict(tx_theta=tx[:N], rx_theta=rx, rx_num=num, rx_den=den, pairs=pairs, S=s_out.value,
                compression=comp.value)


def build_luts(g: Geom, gr: Grid, tx_theta, rx_theta) -> dict:
    tx = np.ascontiguousarray(tx_theta, dtype=np.float64)
    rx = np.ascontiguousarray(rx_theta, dtype=np.float64)
    N, M = len(tx), len(rx)
    l1 = np.zeros((N, gr.X), np.int32)
    l2 = np.zeros((N, gr.Z), np.int32)
    l3 = np.zeros((M, gr.X), np.int32)
    l4 = np.zeros((M, gr.Z), np.int32)
    sh = np.zeros((M, g.L), np.int32)
    t0, tp = _i32(0), _i32(0)
    st = lib().kk_build_luts(ctypes.byref(g), ctypes.byref(gr), _dpp(tx), N, _dpp(rx), M, _ip(l1), _ip(l2),
                             _ip(l3), _ip(l4), ctypes.byref(t0), _ip(sh), ctypes.byref(tp))
    _check("kk_build_luts", st)
    return dict(lut1=l1, lut2=l2, lut3=l3, lut4=l4, t0_q=t0.value, shift=sh, tpad=tp.value)


def build_das_rx(g: Geom, gr: Grid) -> np.ndarray:
    rx = np.zeros((gr.X, g.L, gr.Z), np.int32)
    _check("kk_build_das_rx", lib().kk_build_das_rx(ctypes.byref(g), ctypes.byref(gr), _ip(rx)))
    return rx


def beamform_plan(pairs, S: int, N: int, M: int, T: int, luts: dict, gr: Grid) -> np.ndarray:
    pr = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 3)
    arr = [np.ascontiguousarray(luts[k], dtype=np.int32) for k in ("lut1", "lut2", "lut3", "lut4")]
    need = _sz(0)
    args = [_ip(pr), len(pr), S, N, M, T, *[_ip(a) for a in arr], int(luts["t0_q"]), ctypes.byref(gr)]
    st = lib().kk_beamform_plan(*args, None, 0, ctypes.byref(need))
    if st != KK_E_CAPACITY:
        _check("kk_beamform_plan", st)
    plan = np.zeros(need.value // 4, dtype=np.int32)
    _check("kk_beamform_plan", lib().kk_beamform_plan(*args, plan.ctypes.data_as(_vp), plan.nbytes,
                                                      ctypes.byref(need)))
    return plan


def das_plan(N: int, g: Geom, luts: dict, das_rx: np.ndarray, gr: Grid) -> np.ndarray:
    l1 = np.ascontiguousarray(luts["lut1"], dtype=np.int32)
    l2 = np.ascontiguousarray(luts["lut2"], dtype=np.int32)
    rx = np.ascontiguousarray(das_rx, dtype=np.int32)
    need = _sz(0)
    args = [N, ctypes.byref(g), _ip(l1), _ip(l2), _ip(rx), int(luts["t0_q"]), ctypes.byref(gr)]
    st = lib().das_plan(*args, None, 0, ctypes.byref(need))
    if st != KK_E_CAPACITY:
        _check("das_plan", st)
    plan = np.zeros(need.value // 4, dtype=np.int32)
    _check("das_plan", lib().das_plan(*args, plan.ctypes.data_as(_vp), plan.nbytes, ctypes.byref(need)))
    return plan


# --------------------------------------------------------------------------- device calls

def decompose_workspace_bytes(g: Geom, N: int, M: int, tpad: int, precision: int = PREC_FP32) -> int:
    return int(lib().kk_decompose_workspace_bytes(ctypes.byref(g), N, M, tpad, precision))


def decompose(rf, g: Geom, shift_q, M: int, tpad: int, out=None, ws=None, precision: int = PREC_FP32,
              stream=None):
    """rf int16 [N][L][T] and shift_q int32 [M][L] on the device -> complex64 [N][M][T]."""
    N = rf.shape[0]
    if out is None:
        out = torch.empty((N, M, g.T), dtype=torch.complex64, device=rf.device)
    nbytes = decompose_workspace_bytes(g, N, M, tpad, precision)
    if ws is None:
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=rf.device)
    st = lib().kk_decompose(_dev(rf), N, ctypes.byref(g), _dev(shift_q), M, tpad, precision, _dev(out),
                            _dev(ws), ws.numel() * ws.element_size(), _stream(stream))
    _check("kk_decompose", st)
    return out


def beamform_workspace_bytes(plan_host: np.ndarray) -> int:
    return int(lib().kk_beamform_workspace_bytes(plan_host.ctypes.data_as(_vp), plan_host.nbytes))


def beamform(rf_theta, plan_host: np.ndarray, plan_dev, image=None, intensity=None,
             mode: int = COMPOUND_COHERENT, ws=None, stream=None):
    """rf_theta complex64 [N][M][T] -> per-set images complex64 [S][X][Z] (and intensity)."""
    N, M, T = rf_theta.shape
    S, X, Z = int(plan_host[6]), int(plan_host[7]), int(plan_host[8])
    if image is None:
        image = torch.empty((S, X, Z), dtype=torch.complex64, device=rf_theta.device)
    need = beamform_workspace_bytes(plan_host)
    if ws is None and need > 0:
        ws = torch.empty(need, dtype=torch.uint8, device=rf_theta.device)
    st = lib().kk_beamform(_dev(rf_theta), N, M, T, plan_host.ctypes.data_as(_vp), _dev(plan_dev),
                           plan_host.nbytes, _dev(image), _dev(intensity) if intensity is not None else None,
                           mode, _dev(ws) if ws is not None else None,
                           ws.numel() * ws.element_size() if ws is not None else 0, _stream(stream))
    _check("kk_beamform", st)
    return image


def compound(image, mode: int = COMPOUND_COHERENT, out=None, stream=None):
    S, X, Z = image.shape
    if out is None:
        out = torch.empty((X, Z), dtype=torch.float32, device=image.device)
    _check("kk_compound", lib().kk_compound(_dev(image), S, X, Z, mode, _dev(out), _stream(stream)))
    return out


def das_workspace_bytes(g: Geom, N: int, plan_host: np.ndarray) -> int:
    return int(lib().das_workspace_bytes(ctypes.byref(g), N, plan_host.ctypes.data_as(_vp), plan_host.nbytes))


def das_beamform(rf, g: Geom, plan_host: np.ndarray, plan_dev, image=None, ws=None, stream=None):
    N = rf.shape[0]
    X, Z = int(plan_host[7]), int(plan_host[8])
    if image is None:
        image = torch.empty((X, Z), dtype=torch.complex64, device=rf.device)
    nbytes = das_workspace_bytes(g, N, plan_host)
    if ws is None:
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=rf.device)
    st = lib().das_beamform(_dev(rf), N, ctypes.byref(g), plan_host.ctypes.data_as(_vp), _dev(plan_dev),
                            plan_host.nbytes, _dev(image), _dev(ws), ws.numel() * ws.element_size(),
                            _stream(stream))
    _check("das_beamform", st)
    return image


def to_device(a: np.ndarray, device="cuda"):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device)


@dataclass
class Setup:
    """Per-geometry state of one acquisition: angles, tables and plans (host) plus their
    device copies.  Built once; frames reuse it."""
    geom: Geom
    grid: Grid
    sel: dict
    luts: dict
    plan: np.ndarray
    N: int
    M: int
    T: int
    tpad: int
    das_plan: np.ndarray | None = None


def make_setup(w, with_das: bool = False, scheme=None, M=None, j_list=None) -> Setup:
    """Selection, tables and plans for a configs.Workload."""
    g = geom(w.L, w.T, w.pitch, w.c, w.fs, w.t0)
    gr = grid(w.X, w.Z, w.x0, w.dx, w.z0, w.dz)
    sel = select_pairs(w.scheme if scheme is None else scheme, w.L, w.N, w.theta_max,
                       w.M if M is None else M, w.j_list if j_list is None else j_list)
    luts = build_luts(g, gr, sel["tx_theta"], sel["rx_theta"])
    Md = len(sel["rx_theta"])
    plan = beamform_plan(sel["pairs"], sel["S"], w.N, Md, w.T, luts, gr)
    dp = None
    if with_das:
        dp = das_plan(w.N, g, luts, build_das_rx(g, gr), gr)
    return Setup(g, gr, sel, luts, plan, w.N, Md, w.T, luts["tpad"], dp)
