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

STAGE_FFT, STAGE_CONTRACT, STAGE_INVERSE, STAGE_GATHER, STAGE_REDUCE, STAGE_ALL = 1, 2, 4, 8, 16, 31
ENSEMBLE_CLASSES = 8
WINDOW_CLASSES = (64, 128, 192, 256, 320, 384, 448, 512)

EXPORTS = [
    "kk_select_pairs", "kk_build_luts", "kk_build_das_rx", "kk_beamform_plan",
    "kk_decompose_workspace_bytes", "kk_decompose", "kk_decompose_prepare", "kk_decompose_prepared",
    "kk_beamform_workspace_bytes", "kk_beamform",
    "kk_compound", "das_plan", "das_workspace_bytes", "das_beamform", "kk_status_string",
    "kk_ensemble_default_tuning", "kk_ensemble_plan", "kk_ensemble_query", "kk_ensemble_frame_query",
    "kk_ensemble_run", "kk_ensemble_graph_create", "kk_ensemble_graph_launch", "kk_ensemble_graph_destroy",
    "kk_ensemble_autotune",
    "kk_spectrum_bins", "kk_decompose_spectrum", "kk_spectrum_inverse",
    "kk_net_param_count", "kk_net_state_bytes", "kk_net_workspace_bytes", "kk_net_load", "kk_net_read",
    "kk_net_prepare", "kk_net_forward", "kk_net_backward", "kk_net_adam", "kk_net_train_step", "kk_net_merge",
    "kk_clear", "kk_beamform_static", "kk_beamform_static_max_bytes",
]
# plan header words (the PlanWord order of the library's plan format): window class, pair shares
PLAN_WORD_CAP, PLAN_WORD_SPLIT = 13, 24
NET_LAYERS, NET_WIDTH, NET_IN = 6, 32, 8
NET_PARAMS, NET_GRADS, NET_MOMENT1, NET_MOMENT2 = 0, 1, 2, 3


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


class EnsembleFrame(ctypes.Structure):
    _fields_ = [("geom", Geom), ("N", ctypes.c_int32), ("M", ctypes.c_int32), ("tpad", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("shift_q", ctypes.c_void_p), ("plan", ctypes.c_void_p),
                ("plan_bytes", ctypes.c_size_t)]


class EnsembleTuning(ctypes.Structure):
    _fields_ = [("pair_tile", ctypes.c_int32 * ENSEMBLE_CLASSES), ("queue", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 7)]

    def as_dict(self) -> dict:
        return dict(pair_tile={WINDOW_CLASSES[c]: int(self.pair_tile[c]) for c in range(ENSEMBLE_CLASSES)},
                    queue=int(self.queue))


class EnsembleFrameInfo(ctypes.Structure):
    _fields_ = [("rf_offset", ctypes.c_int64), ("image_offset", ctypes.c_int64),
                ("intensity_offset", ctypes.c_int64), ("rf_theta_offset", ctypes.c_int64),
                ("share_offset", ctypes.c_int64)] + \
               [(n, ctypes.c_int32) for n in ("N", "L", "T", "M", "S", "X", "Z", "P", "tpad", "cap", "split",
                                               "group", "mode", "plan_offset", "shift_offset", "reserved")]


class EnsembleSizes(ctypes.Structure):
    _fields_ = [("rf_elems", ctypes.c_int64), ("image_elems", ctypes.c_int64),
                ("intensity_elems", ctypes.c_int64), ("ws_bytes", ctypes.c_int64),
                ("units_offset", ctypes.c_int64), ("nframes", ctypes.c_int32), ("ngroups", ctypes.c_int32),
                ("nlaunches", ctypes.c_int32), ("nunits", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


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
            "kk_decompose_prepare": [ctypes.POINTER(Geom), _i32, _vp, _i32, _i32, _i32, _vp, _sz, _vp],
            "kk_decompose_prepared": [_vp, _i32, ctypes.POINTER(Geom), _vp, _i32, _i32, _i32, _vp, _vp, _sz, _vp],
            "kk_beamform": [_vp, _i32, _i32, _i32, _vp, _vp, _sz, _vp, _vp, _i32, _vp, _sz, _vp],
            "kk_compound": [_vp, _i32, _i32, _i32, _i32, _vp, _vp],
            "das_plan": [_i32, ctypes.POINTER(Geom), _i32p, _i32p, _i32p, _i32, ctypes.POINTER(Grid), _vp, _sz,
                         _szp],
            "das_beamform": [_vp, _i32, ctypes.POINTER(Geom), _vp, _vp, _sz, _vp, _vp, _sz, _vp],
            "kk_ensemble_plan": [ctypes.POINTER(EnsembleFrame), _i32, _i32, ctypes.POINTER(EnsembleTuning),
                                 ctypes.c_int64, _vp, _sz, _szp],
            "kk_ensemble_query": [_vp, _sz, ctypes.POINTER(EnsembleSizes)],
            "kk_ensemble_frame_query": [_vp, _sz, _i32, ctypes.POINTER(EnsembleFrameInfo)],
            "kk_ensemble_run": [_vp, _vp, _sz, _vp, _vp, _vp, _vp, _sz, _i32, _vp],
            "kk_ensemble_graph_create": [_vp, _vp, _sz, _vp, _vp, _vp, _vp, _sz, _vp,
                                         ctypes.POINTER(ctypes.c_void_p)],
            "kk_ensemble_graph_launch": [_vp, _vp],
            "kk_ensemble_graph_destroy": [_vp],
            "kk_spectrum_bins": [_i32],
            "kk_decompose_spectrum": [_vp, _i32, ctypes.POINTER(Geom), _vp, _i32, _i32, _i32, _vp, _vp, _sz, _vp],
            "kk_spectrum_inverse": [_vp, _i32, _i32, _i32, _vp, _vp],
            "kk_net_load": [_vp, _vp, _vp],
            "kk_net_read": [_vp, _i32, _vp, _vp],
            "kk_net_prepare": [_vp, _i32, _i32, _i32, _vp, _i32, _i32, _vp, _i32, _vp, _i32, _vp, _vp, _vp, _vp],
            "kk_net_forward": [_vp, _vp, _vp, _i32, _i32, _i32, _i32p, _vp, _vp, _sz, _vp],
            "kk_net_backward": [_vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32p, ctypes.c_float, _vp, _vp, _sz, _vp],
            "kk_net_adam": [_vp, _i32, ctypes.c_float, _vp],
            "kk_net_train_step": [_vp, _vp, _vp, _vp, _i32, _i32, _i32, _i32p, ctypes.c_float, _i32, ctypes.c_float,
                                  _vp, _vp, _sz, _vp],
            "kk_net_merge": [_vp, _vp, _vp, _i32, _i32, _vp, _i32, _i32, _i32, _vp, _vp, _i32, _vp, _vp],
            "kk_clear": [_vp, _sz, _vp],
            "kk_beamform_static": [_vp, _i32, _i32, _i32, _vp, _vp, _sz, _vp, _vp, _i32, _vp],
            "kk_ensemble_autotune": [ctypes.POINTER(EnsembleFrame), _i32, _i32, ctypes.c_int64, _vp, _sz, _vp, _vp,
                                     _vp, _vp, _sz, _i32, _vp, ctypes.POINTER(EnsembleTuning),
                                     ctypes.POINTER(ctypes.c_float)],
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
        L.kk_beamform_static_max_bytes.argtypes = []
        L.kk_beamform_static_max_bytes.restype = _sz
        for name in ("kk_net_param_count", "kk_net_state_bytes"):
            getattr(L, name).argtypes = []
            getattr(L, name).restype = _sz
        L.kk_net_workspace_bytes.argtypes = [_i32, _i32, _i32]
        L.kk_net_workspace_bytes.restype = _sz
        L.kk_ensemble_default_tuning.argtypes = [ctypes.POINTER(EnsembleTuning)]
        L.kk_ensemble_default_tuning.restype = None
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


def _bind(stream, *allocated):
    """Tensors this module allocated for a call on an explicit stream are marked as used by
    that stream, so that torch's caching allocator does not hand their memory to another
    allocation before the enqueued kernels have finished with it."""
    if stream is None:
        return
    s = stream if isinstance(stream, torch.cuda.Stream) else torch.cuda.ExternalStream(_stream(stream))
    for t in allocated:
        if t is not None:
            t.record_stream(s)


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
              stream=None, prepared: bool = False):
    """rf int16 [N][L][T] and shift_q int32 [M][L] on the device -> complex64 [N][M][T].
    prepared: ws was prepared by decompose_prepare for this geometry (kk_decompose_prepared)."""
    N = rf.shape[0]
    new = []
    if out is None:
        out = torch.empty((N, M, g.T), dtype=torch.complex64, device=rf.device)
        new.append(out)
    nbytes = decompose_workspace_bytes(g, N, M, tpad, precision)
    if ws is None:
        if prepared:
            raise ValueError("a prepared decomposition needs its prepared workspace")
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=rf.device)
        new.append(ws)
    name = "kk_decompose_prepared" if prepared else "kk_decompose"
    st = getattr(lib(), name)(_dev(rf), N, ctypes.byref(g), _dev(shift_q), M, tpad, precision, _dev(out),
                              _dev(ws), ws.numel() * ws.element_size(), _stream(stream))
    _bind(stream, *new)
    _check(name, st)
    return out


def decompose_prepare(g: Geom, N: int, shift_q, M: int, tpad: int, ws, precision: int = PREC_FP32, stream=None):
    """Writes the phase tables of (g, N, shift_q, M, tpad) into ws (kk_decompose_prepare)."""
    st = lib().kk_decompose_prepare(ctypes.byref(g), N, _dev(shift_q), M, tpad, precision, _dev(ws),
                                    ws.numel() * ws.element_size(), _stream(stream))
    _check("kk_decompose_prepare", st)
    return ws


def beamform_workspace_bytes(plan_host: np.ndarray) -> int:
    return int(lib().kk_beamform_workspace_bytes(plan_host.ctypes.data_as(_vp), plan_host.nbytes))


def beamform(rf_theta, plan_host: np.ndarray, plan_dev, image=None, intensity=None,
             mode: int = COMPOUND_COHERENT, ws=None, stream=None):
    """rf_theta complex64 [N][M][T] -> per-set images complex64 [S][X][Z] (and intensity)."""
    N, M, T = rf_theta.shape
    S, X, Z = int(plan_host[6]), int(plan_host[7]), int(plan_host[8])
    new = []
    if image is None:
        image = torch.empty((S, X, Z), dtype=torch.complex64, device=rf_theta.device)
        new.append(image)
    need = beamform_workspace_bytes(plan_host)
    if ws is None and need > 0:
        ws = torch.empty(need, dtype=torch.uint8, device=rf_theta.device)
        new.append(ws)
    st = lib().kk_beamform(_dev(rf_theta), N, M, T, plan_host.ctypes.data_as(_vp), _dev(plan_dev),
                           plan_host.nbytes, _dev(image), _dev(intensity) if intensity is not None else None,
                           mode, _dev(ws) if ws is not None else None,
                           ws.numel() * ws.element_size() if ws is not None else 0, _stream(stream))
    _bind(stream, *new)
    _check("kk_beamform", st)
    return image


def beamform_static_max_bytes() -> int:
    return int(lib().kk_beamform_static_max_bytes())


def beamform_static(rf_theta, plan_host: np.ndarray, plan_dev, image, intensity=None,
                    mode: int = COMPOUND_COHERENT, stream=None):
    """kk_beamform without a workspace (see kk_beamform_static): the caller passes the outputs."""
    N, M, T = rf_theta.shape
    st = lib().kk_beamform_static(_dev(rf_theta), N, M, T, plan_host.ctypes.data_as(_vp), _dev(plan_dev),
                                  plan_host.nbytes, _dev(image), _dev(intensity) if intensity is not None else None,
                                  mode, _stream(stream))
    _check("kk_beamform_static", st)
    return image


def compound(image, mode: int = COMPOUND_COHERENT, out=None, stream=None):
    S, X, Z = image.shape
    new = None
    if out is None:
        out = new = torch.empty((X, Z), dtype=torch.float32, device=image.device)
    st = lib().kk_compound(_dev(image), S, X, Z, mode, _dev(out), _stream(stream))
    _bind(stream, new)
    _check("kk_compound", st)
    return out


def das_workspace_bytes(g: Geom, N: int, plan_host: np.ndarray) -> int:
    return int(lib().das_workspace_bytes(ctypes.byref(g), N, plan_host.ctypes.data_as(_vp), plan_host.nbytes))


def das_beamform(rf, g: Geom, plan_host: np.ndarray, plan_dev, image=None, ws=None, stream=None):
    N = rf.shape[0]
    X, Z = int(plan_host[7]), int(plan_host[8])
    new = []
    if image is None:
        image = torch.empty((X, Z), dtype=torch.complex64, device=rf.device)
        new.append(image)
    nbytes = das_workspace_bytes(g, N, plan_host)
    if ws is None:
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=rf.device)
        new.append(ws)
    st = lib().das_beamform(_dev(rf), N, ctypes.byref(g), plan_host.ctypes.data_as(_vp), _dev(plan_dev),
                            plan_host.nbytes, _dev(image), _dev(ws), ws.numel() * ws.element_size(),
                            _stream(stream))
    _bind(stream, *new)
    _check("das_beamform", st)
    return image


def spectrum_bins(tpad: int) -> int:
    return int(lib().kk_spectrum_bins(tpad))


def decompose_spectrum(rf, g: Geom, shift_q, M: int, tpad: int, out=None, ws=None, precision: int = PREC_FP32,
                       stream=None):
    """rf int16 [N][L][T], shift_q int32 [M][L] on the device -> complex64 [N][M][kpad] (bins >= tpad/2 zero)."""
    N = rf.shape[0]
    kpad = spectrum_bins(tpad)
    new = []
    if out is None:
        out = torch.empty((N, M, kpad), dtype=torch.complex64, device=rf.device)
        new.append(out)
    nbytes = decompose_workspace_bytes(g, N, M, tpad, precision)
    if ws is None:
        ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=rf.device)
        new.append(ws)
    st = lib().kk_decompose_spectrum(_dev(rf), N, ctypes.byref(g), _dev(shift_q), M, tpad, precision, _dev(out),
                                     _dev(ws), ws.numel() * ws.element_size(), _stream(stream))
    _bind(stream, *new)
    _check("kk_decompose_spectrum", st)
    return out


def spectrum_inverse(spec, tpad: int, T: int, out=None, stream=None):
    """spec complex64 [..., kpad] -> complex64 [..., T] (first T samples of the inverse transform)."""
    lead = spec.shape[:-1]
    n = int(np.prod(lead))
    new = None
    if out is None:
        out = new = torch.empty(tuple(lead) + (T,), dtype=torch.complex64, device=spec.device)
    st = lib().kk_spectrum_inverse(_dev(spec), n, tpad, T, _dev(out), _stream(stream))
    _bind(stream, new)
    _check("kk_spectrum_inverse", st)
    return out


def clear(t, stream=None):
    _check("kk_clear", lib().kk_clear(_dev(t), t.numel() * t.element_size(), _stream(stream)))


def net_param_count() -> int:
    return int(lib().kk_net_param_count())


def net_layer_shapes():
    """[(cin, offset of W, offset of bias)] per layer of the flat FP32 parameter vector."""
    out, off = [], 0
    for l in range(NET_LAYERS):
        cin = NET_IN if l == 0 else NET_WIDTH
        out.append((cin, off, off + 9 * NET_WIDTH * cin))
        off += 9 * NET_WIDTH * cin + NET_WIDTH
    assert off == net_param_count()
    return out


class Net:
    """Device state of the completion network (parameters, Adam moments, gradient, BF16
    weights) and its workspace for batches of up to B grids of H x W."""

    def __init__(self, params: np.ndarray, B: int, H: int, W: int, device="cuda", dilation=None):
        self.B, self.H, self.W = B, H, W
        self.dilation = [(1, 1)] * NET_LAYERS if dilation is None else [tuple(d) for d in dilation]
        self._dil = np.ascontiguousarray(np.array(self.dilation, dtype=np.int32).ravel())
        self.state = torch.zeros(int(lib().kk_net_state_bytes()), dtype=torch.uint8, device=device)
        nb = int(lib().kk_net_workspace_bytes(B, H, W))
        if nb == 0:
            raise ValueError("unsupported grid shape %dx%d" % (H, W))
        self.ws = torch.zeros(nb, dtype=torch.uint8, device=device)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.step = 0
        self.load(params)

    def load(self, params: np.ndarray, stream=None):
        p = np.ascontiguousarray(params, dtype=np.float32)
        if p.size != net_param_count():
            raise ValueError("expected %d parameters" % net_param_count())
        _check("kk_net_load", lib().kk_net_load(_dev(self.state), p.ctypes.data, _stream(stream)))
        self.step = 0

    def read(self, what: int = NET_PARAMS, stream=None) -> np.ndarray:
        out = np.zeros(net_param_count(), dtype=np.float32)
        _check("kk_net_read", lib().kk_net_read(_dev(self.state), what, out.ctypes.data, _stream(stream)))
        return out

    def forward(self, grid, out, B=None, sidx=None, stream=None):
        B = self.B if B is None else B
        _check("kk_net_forward", lib().kk_net_forward(_dev(self.state), _dev(grid), _dev(sidx) if sidx is not None
                                                      else None, B, self.H, self.W, _ip(self._dil), _dev(out),
                                                      _dev(self.ws), self.ws.numel(), _stream(stream)))
        return out

    def backward(self, grid, target, inv_count: float, B=None, sidx=None, stream=None):
        B = self.B if B is None else B
        _check("kk_net_backward", lib().kk_net_backward(_dev(self.state), _dev(grid), _dev(target),
                                                        _dev(sidx) if sidx is not None else None, B, self.H, self.W,
                                                        _ip(self._dil), inv_count, _dev(self.loss), _dev(self.ws),
                                                        self.ws.numel(), _stream(stream)))
        return self.loss

    def adam(self, lr: float, stream=None):
        self.step += 1
        _check("kk_net_adam", lib().kk_net_adam(_dev(self.state), self.step, lr, _stream(stream)))

    def train_step(self, grid, target, inv_count: float, lr: float, B=None, sidx=None, stream=None):
        B = self.B if B is None else B
        self.step += 1
        _check("kk_net_train_step", lib().kk_net_train_step(_dev(self.state), _dev(grid), _dev(target),
                                                            _dev(sidx) if sidx is not None else None, B, self.H,
                                                            self.W, _ip(self._dil), inv_count, self.step, lr,
                                                            _dev(self.loss), _dev(self.ws), self.ws.numel(),
                                                            _stream(stream)))
        return self.loss


def net_prepare(spec, obs_src, grid_to_obs, grid, scale, bins=None, k_first: int = 0, B=None, target=None,
                stream=None):
    """Input grids (and targets) from spec complex64 [H][Msrc][kpad] (see kk_net_prepare)."""
    H, Msrc, kpad = spec.shape
    W = grid_to_obs.numel()
    B = (bins.numel() if bins is not None else grid.shape[0]) if B is None else B
    _check("kk_net_prepare", lib().kk_net_prepare(_dev(spec), H, Msrc, kpad, _dev(bins) if bins is not None else None,
                                                  k_first, B, _dev(obs_src), obs_src.numel(), _dev(grid_to_obs), W,
                                                  _dev(grid), _dev(target) if target is not None else None,
                                                  _dev(scale), _stream(stream)))


def net_merge(out, scale, spec, obs_src, grid_to_obs, dst, bins=None, k_first: int = 0, B=None, stream=None):
    H, Msrc, kpad = spec.shape
    W = grid_to_obs.numel()
    B = (bins.numel() if bins is not None else out.shape[0]) if B is None else B
    _check("kk_net_merge", lib().kk_net_merge(_dev(out), _dev(scale), _dev(bins) if bins is not None else None,
                                              k_first, B, _dev(spec), H, Msrc, kpad, _dev(obs_src),
                                              _dev(grid_to_obs), W, _dev(dst), _stream(stream)))


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


# --------------------------------------------------------------------------- frame ensembles

def default_tuning() -> EnsembleTuning:
    t = EnsembleTuning()
    lib().kk_ensemble_default_tuning(ctypes.byref(t))
    return t


@dataclass
class EnsembleInput:
    """One frame of an ensemble: its geometry, angle counts, shear table and beamforming plan
    (host arrays from build_luts / beamform_plan) and the intensity mode (-1: none)."""
    geom: Geom
    N: int
    M: int
    tpad: int
    shift: np.ndarray
    plan: np.ndarray
    mode: int = COMPOUND_INCOHERENT


def setup_frame_input(su: "Setup", mode: int = COMPOUND_INCOHERENT) -> EnsembleInput:
    return EnsembleInput(su.geom, su.N, su.M, su.tpad, np.ascontiguousarray(su.luts["shift"], dtype=np.int32),
                         np.ascontiguousarray(su.plan, dtype=np.int32), mode)


class Ensemble:
    """A planned frame ensemble and its packed device buffers (channel data in, images and
    intensities out, workspace).  frame_rf(f) / frame_image(f) / frame_intensity(f) are views
    of frame f's slices."""

    def __init__(self, inputs, precision: int = PREC_BF16X3, tuning: EnsembleTuning | None = None,
                 spectra_budget: int = 0, device="cuda", allocate: bool = True):
        self.inputs = list(inputs)
        self.precision = precision
        self.spectra_budget = int(spectra_budget)
        self._keep = [(np.ascontiguousarray(x.shift, dtype=np.int32), np.ascontiguousarray(x.plan, dtype=np.int32))
                      for x in self.inputs]
        arr = (EnsembleFrame * len(self.inputs))()
        for i, (x, (sh, pl)) in enumerate(zip(self.inputs, self._keep)):
            arr[i] = EnsembleFrame(x.geom, x.N, x.M, x.tpad, x.mode, sh.ctypes.data, pl.ctypes.data, pl.nbytes)
        self._frames = arr
        self.tuning = tuning if tuning is not None else default_tuning()
        self.device = device
        self.plan_dev = None
        self._plan()
        if allocate:
            self.allocate()

    def _plan(self):
        need = _sz(0)
        args = [self._frames, len(self.inputs), self.precision, ctypes.byref(self.tuning), self.spectra_budget]
        st = lib().kk_ensemble_plan(*args, None, 0, ctypes.byref(need))
        if st != KK_E_CAPACITY:
            _check("kk_ensemble_plan", st)
        plan = np.zeros(need.value // 4, dtype=np.int32)
        _check("kk_ensemble_plan", lib().kk_ensemble_plan(*args, plan.ctypes.data_as(_vp), plan.nbytes,
                                                          ctypes.byref(need)))
        self.plan_host = plan
        self.sizes = EnsembleSizes()
        _check("kk_ensemble_query", lib().kk_ensemble_query(plan.ctypes.data_as(_vp), plan.nbytes,
                                                            ctypes.byref(self.sizes)))
        self.info = []
        for f in range(len(self.inputs)):
            fi = EnsembleFrameInfo()
            _check("kk_ensemble_frame_query", lib().kk_ensemble_frame_query(plan.ctypes.data_as(_vp), plan.nbytes,
                                                                            f, ctypes.byref(fi)))
            self.info.append(fi)

    def allocate(self):
        dev = self.device
        s = self.sizes
        self.rf = torch.zeros(max(int(s.rf_elems), 1), dtype=torch.int16, device=dev)
        self.image = torch.zeros(max(int(s.image_elems), 1), dtype=torch.complex64, device=dev)
        self.intensity = torch.zeros(max(int(s.intensity_elems), 1), dtype=torch.float32, device=dev)
        self.ws = torch.zeros(max(int(s.ws_bytes), 1), dtype=torch.uint8, device=dev)
        self.upload_plan()

    def upload_plan(self):
        if self.plan_dev is None or self.plan_dev.numel() < self.plan_host.size:
            self.plan_dev = to_device(self.plan_host, self.device)
        else:
            self.plan_dev[: self.plan_host.size].copy_(torch.from_numpy(self.plan_host))

    def retune(self, tuning: EnsembleTuning):
        """Re-plan with new launch shapes (same frames), reallocating what grew."""
        self.tuning = tuning
        old_ws = self.ws.numel()
        self._plan()
        if int(self.sizes.ws_bytes) > old_ws:
            self.ws = torch.zeros(int(self.sizes.ws_bytes), dtype=torch.uint8, device=self.device)
        self.upload_plan()

    # views
    def frame_rf(self, f):
        i = self.info[f]
        n = i.N * i.L * i.T
        return self.rf[i.rf_offset: i.rf_offset + n].view(i.N, i.L, i.T)

    def frame_image(self, f):
        i = self.info[f]
        n = i.S * i.X * i.Z
        return self.image[i.image_offset: i.image_offset + n].view(i.S, i.X, i.Z)

    def frame_intensity(self, f):
        i = self.info[f]
        if i.intensity_offset < 0:
            return None
        return self.intensity[i.intensity_offset: i.intensity_offset + i.X * i.Z].view(i.X, i.Z)

    def frame_rf_theta(self, f):
        i = self.info[f]
        n = i.N * i.M * i.T
        b = i.rf_theta_offset * 8
        return self.ws[b: b + n * 8].view(torch.complex64).view(i.N, i.M, i.T)

    def unit_counts(self) -> np.ndarray:
        """Per window class and workgroup: gather units taken in the last run [8][1024]."""
        b = int(self.sizes.units_offset)
        return self.ws[b: b + ENSEMBLE_CLASSES * 1024 * 4].view(torch.int32).view(ENSEMBLE_CLASSES, 1024).cpu().numpy()

    def _bufs(self):
        return (self.plan_host.ctypes.data_as(_vp), _dev(self.plan_dev), self.plan_host.nbytes, _dev(self.rf),
                _dev(self.image), _dev(self.intensity), _dev(self.ws), self.ws.numel())

    def run(self, stages: int = STAGE_ALL, stream=None):
        _check("kk_ensemble_run", lib().kk_ensemble_run(*self._bufs(), stages, _stream(stream)))

    def graph(self, stream) -> "EnsembleGraph":
        h = ctypes.c_void_p(0)
        _check("kk_ensemble_graph_create", lib().kk_ensemble_graph_create(*self._bufs(), _stream(stream),
                                                                          ctypes.byref(h)))
        return EnsembleGraph(h)

    def autotune(self, reps: int = 3, stream=None):
        """Measure launch shapes on the device (synchronous); re-plans with the best and returns
        (tuning, gather + reduce microseconds).  The candidate plans and workspace are sized for
        the largest pair split (8 shares per set), so that every candidate fits."""
        t = EnsembleTuning()
        ctypes.memmove(ctypes.byref(t), ctypes.byref(self.tuning), ctypes.sizeof(t))
        us = ctypes.c_float(0)
        units = sum(((i.X + 63) // 64) * ((i.Z + 15) // 16) * i.S for i in self.info)
        plan_cap = self.plan_host.nbytes + 8 * 8 * units + (1 << 16)
        scratch = torch.empty((plan_cap + 3) // 4, dtype=torch.int32, device=self.device)
        ws_need = int(self.sizes.ws_bytes) + sum(8 * 8 * i.S * i.X * i.Z + 256 for i in self.info)
        if self.ws.numel() < ws_need:
            self.ws = torch.zeros(ws_need, dtype=torch.uint8, device=self.device)
        _check("kk_ensemble_autotune",
               lib().kk_ensemble_autotune(self._frames, len(self.inputs), self.precision, self.spectra_budget,
                                          _dev(scratch), plan_cap, _dev(self.rf), _dev(self.image),
                                          _dev(self.intensity), _dev(self.ws), self.ws.numel(), reps,
                                          _stream(stream), ctypes.byref(t), ctypes.byref(us)))
        del scratch
        self.retune(t)
        return t, float(us.value)


class EnsembleGraph:
    def __init__(self, handle):
        self.handle = handle

    def launch(self, stream):
        _check("kk_ensemble_graph_launch", lib().kk_ensemble_graph_launch(self.handle, _stream(stream)))

    def destroy(self):
        if self.handle:
            _check("kk_ensemble_graph_destroy", lib().kk_ensemble_graph_destroy(self.handle))
            self.handle = None
