"""ctypes binding of libvelo.so (include/velo.h).

Argument marshalling only: buffers are torch tensors on a ROCm device (used
for device memory and streams), every computation runs in the library's HIP
kernels.  There is no CPU fallback: a missing library raises.

Unsigned device data are carried in signed torch dtypes of the same width
(uint32 -> int32, uint64 -> int64); use `.view(torch.uint32)` style
reinterpretation or numpy `.view(np.uint32)` on the host to read them.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libvelo.so")

EV_BAD_WORD = 1
EV_LAYER_ORDER = 2
EV_DUPLICATE = 4
EV_HOLE = 8
EV_OVERFLOW = 16
EV_BAD_OFFSETS = 32
MAX_CANDIDATES = 65536
N_LAYERS = 26


class VeloError(RuntimeError):
    pass


class Params(C.Structure):
    _fields_ = [("max_t", C.c_float), ("sin2_phi", C.c_float), ("s_seed", C.c_float),
                ("s_fwd", C.c_float), ("max_skip", C.c_int32), ("sigma_meas", C.c_float),
                ("pt0_mev", C.c_float), ("x_over_x0", C.c_float), ("qc3", C.c_float),
                ("qc4", C.c_float)]


class Geometry(C.Structure):
    _fields_ = [("n_layers", C.c_int32), ("z_mm", C.c_float * 26), ("pitch_mm", C.c_float),
                ("n_cols", C.c_int32), ("n_rows", C.c_int32), ("hole_r_mm", C.c_float)]


class _Hits(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "key", "aux", "layer_start", "layer_nhits",
                                           "n_hits", "status")]


class _Tracks(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("n_tracks", "nhits", "hit_idx", "status")]


class _States(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("x", "y", "z", "tx", "ty", "cov_x", "cov_y", "chi2",
                                           "ndof", "accepted", "score")]


class _Mlp(C.Structure):
    _fields_ = [("params", C.c_void_p), ("mean", C.c_void_p), ("std", C.c_void_p),
                ("threshold", C.c_float)]


N_FEATURES = 8
N_PARAMS = 1377


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded libvelo.so (raises VeloError when it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise VeloError(f"{_LIB_PATH} is missing: build it with paper_1912_09161_amd/build.py")
        L = C.CDLL(_LIB_PATH)
        P = C.c_void_p
        L.velo_params_default.argtypes = [P]
        L.velo_params_default.restype = None
        L.velo_geometry_default.argtypes = [P]
        L.velo_geometry_default.restype = None
        L.velo_workspace_bytes.argtypes = [C.c_uint64, C.c_uint32]
        L.velo_workspace_bytes.restype = C.c_size_t
        L.velo_cluster.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, P, C.c_size_t, P]
        L.velo_cluster.restype = C.c_int
        L.velo_find_tracks.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, P, P, C.c_size_t, P]
        L.velo_find_tracks.restype = C.c_int
        L.velo_fit.argtypes = [P, P, P, C.c_uint32, C.c_uint64, P, P, P, P]
        L.velo_fit.restype = C.c_int
        L.velo_fit_momentum.argtypes = [P, P, P, C.c_uint32, C.c_uint64, P, P, P, P, P]
        L.velo_fit_momentum.restype = C.c_int
        L.velo_ut_params_default.argtypes = [P]
        L.velo_ut_params_default.restype = None
        L.velo_ut_windows.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, P, C.c_uint64, P, P, P]
        L.velo_ut_windows.restype = C.c_int
        L.velo_reconstruct.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, P, P, P, P, C.c_size_t, P]
        L.velo_reconstruct.restype = C.c_int
        L.velo_reconstruct_noalloc.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, P, P, P, P]
        L.velo_reconstruct_noalloc.restype = C.c_int
        L.velo_pv_params_default.argtypes = [P]
        L.velo_pv_params_default.restype = None
        L.velo_find_pvs.argtypes = [P, P, P, C.c_uint32, C.c_uint64, P, P, P]
        L.velo_find_pvs.restype = C.c_int
        L.velo_pipeline_create.argtypes = [P, P, P, P, P, P]
        L.velo_pipeline_create.restype = C.c_int
        L.velo_pipeline_destroy.argtypes = [P]
        L.velo_pipeline_destroy.restype = None
        L.velo_pipeline_run.argtypes = [P, P, C.c_uint64, P, C.c_uint32, P, P]
        L.velo_pipeline_run.restype = C.c_int
        L.velo_reconstruct_timed.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, P, P, P, P, C.c_size_t, P, P]
        L.velo_reconstruct_timed.restype = C.c_int
        L.velo_mlp_load.argtypes = [P, P, C.c_size_t]
        L.velo_mlp_load.restype = C.c_int
        L.velo_mlp_save.argtypes = [P, P, C.c_size_t]
        L.velo_mlp_save.restype = C.c_int
        L.velo_mlp_train_step.argtypes = [P, P, P, P, C.c_uint32, C.c_float, C.c_uint32, P, P]
        L.velo_mlp_train_step.restype = C.c_int
        L.velo_check_status.argtypes = [P, P, C.c_uint32, P, P, P]
        L.velo_check_status.restype = C.c_int
        L.velo_status_string.argtypes = [C.c_int]
        L.velo_status_string.restype = C.c_char_p
        L.velo_fit_mlp.argtypes = [P, P, P, C.c_uint32, C.c_uint64, P, P, P, P, P]
        L.velo_fit_mlp.restype = C.c_int
        L.velo_reconstruct_mlp.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, P, P, P, P, P, C.c_size_t, P]
        L.velo_reconstruct_mlp.restype = C.c_int
        L.velo_track_features.argtypes = [P, P, P, P, C.c_uint32, C.c_uint64, P, P, P]
        L.velo_track_features.restype = C.c_int
        L.velo_mlp_workspace_bytes.argtypes = [C.c_uint32]
        L.velo_mlp_workspace_bytes.restype = C.c_size_t
        L.velo_feature_stats.argtypes = [P, C.c_uint64, P, P, P, C.c_size_t, P]
        L.velo_feature_stats.restype = C.c_int
        L.velo_mlp_fwd_bwd.argtypes = [P, P, P, P, P, P, C.c_uint32, P, P, P, C.c_size_t, P]
        L.velo_mlp_fwd_bwd.restype = C.c_int
        L.velo_mlp_adam_step.argtypes = [P, P, P, P, C.c_uint32, C.c_float, P]
        L.velo_mlp_adam_step.restype = C.c_int
        L.velo_mlp_infer.argtypes = [P, P, C.c_uint32, P, P]
        L.velo_mlp_infer.restype = C.c_int
        L.velo_context_create.argtypes = [P, P, P]
        L.velo_context_create.restype = C.c_int
        L.velo_context_destroy.argtypes = [P]
        L.velo_context_destroy.restype = None
        L.velo_context_config.argtypes = [P, P, P]
        L.velo_context_config.restype = C.c_int
        L.velo_context_set_config.argtypes = [P, P]
        L.velo_context_set_config.restype = C.c_int
        L.velo_batched_workspace_bytes.argtypes = [C.c_uint64, C.c_uint32]
        L.velo_batched_workspace_bytes.restype = C.c_size_t
        L.velo_reconstruct_batched.argtypes = [P, P, P, C.c_uint32, C.c_uint64, P, P, P, P, P, P,
                                               C.c_size_t, P]
        L.velo_reconstruct_batched.restype = C.c_int
        _lib = L
    return _lib


_GEOM = None


def default_geometry() -> Geometry:
    """The detector model the kernels are built for (velo_geometry_default)."""
    g = Geometry()
    lib().velo_geometry_default(C.byref(g))
    return g


def _geom(g=None):
    global _GEOM
    if g is not None:
        return C.byref(g)
    if _GEOM is None:
        _GEOM = default_geometry()
    return C.byref(_GEOM)


def default_params(**overrides) -> Params:
    p = Params()
    lib().velo_params_default(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def _check(rc: int):
    if rc != 0:
        raise VeloError(f"libvelo: {lib().velo_status_string(rc).decode()} ({rc})")


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def workspace_bytes(n_pixels: int, n_events: int) -> int:
    return int(lib().velo_workspace_bytes(int(n_pixels), int(n_events)))


def alloc_workspace(n_pixels: int, n_events: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(workspace_bytes(n_pixels, n_events), 1), dtype=torch.uint8, device=device)


def alloc_hits(n_pixels: int, n_events: int, device="cuda") -> dict:
    N = max(int(n_pixels), 1)
    E = max(int(n_events), 1)
    f = lambda n, dt: torch.empty(n, dtype=dt, device=device)  # noqa: E731
    return dict(x=f(N, torch.float32), y=f(N, torch.float32), key=f(N, torch.int32),
                aux=f(N, torch.int32), layer_start=f(E * 27, torch.int32),
                layer_nhits=f(E * 26, torch.int32), n_hits=f(E, torch.int32),
                status=f(E, torch.int32))


def track_capacity(n_pixels: int) -> int:
    return max(int(n_pixels) // 3, 1)


def alloc_tracks(n_pixels: int, n_events: int, device="cuda") -> dict:
    cap = track_capacity(n_pixels)
    E = max(int(n_events), 1)
    return dict(n_tracks=torch.empty(E, dtype=torch.int32, device=device),
                nhits=torch.empty(cap, dtype=torch.uint8, device=device),
                hit_idx=torch.empty(cap * 26, dtype=torch.int32, device=device),
                status=torch.empty(E, dtype=torch.int32, device=device))


def alloc_states(n_pixels: int, device="cuda") -> dict:
    cap = track_capacity(n_pixels)
    f = lambda n, dt=torch.float32: torch.empty(n, dtype=dt, device=device)  # noqa: E731
    return dict(x=f(cap), y=f(cap), z=f(cap), tx=f(cap), ty=f(cap), cov_x=f(3 * cap),
                cov_y=f(3 * cap), chi2=f(cap), ndof=f(cap, torch.int32),
                accepted=f(cap, torch.uint8), score=f(cap))


def _hits_struct(h):
    return _Hits(*[_ptr(h[k]) for k, _ in _Hits._fields_])


def _tracks_struct(t):
    return _Tracks(*[_ptr(t[k]) for k, _ in _Tracks._fields_])


def _states_struct(s):
    return _States(*[_ptr(s.get(k)) for k, _ in _States._fields_])


def _n_pixels(pixels) -> int:
    return int(pixels.numel())


def cluster(pixels: torch.Tensor, offsets: torch.Tensor, hits=None, ws=None, stream=None) -> dict:
    """velo_cluster: pixels int32[N] (raw uint32 words), offsets int64[E+1] on the GPU."""
    E = offsets.numel() - 1
    N = _n_pixels(pixels)
    hits = hits if hits is not None else alloc_hits(N, E, pixels.device)
    ws = ws if ws is not None else alloc_workspace(N, E, pixels.device)
    hs = _hits_struct(hits)
    _check(lib().velo_cluster(_ptr(pixels), _ptr(offsets), E, N, _geom(), C.byref(hs), _ptr(ws),
                              ws.numel(), _stream(stream)))
    return hits


def find_tracks(hits: dict, offsets: torch.Tensor, n_pixels: int, params=None, tracks=None, ws=None,
                stream=None) -> dict:
    E = offsets.numel() - 1
    params = params if params is not None else default_params()
    tracks = tracks if tracks is not None else alloc_tracks(n_pixels, E, offsets.device)
    ws = ws if ws is not None else alloc_workspace(n_pixels, E, offsets.device)
    hs, ts = _hits_struct(hits), _tracks_struct(tracks)
    _check(lib().velo_find_tracks(C.byref(hs), _ptr(offsets), E, int(n_pixels), _geom(), C.byref(params),
                                  C.byref(ts), _ptr(ws), ws.numel(), _stream(stream)))
    return tracks


def fit(hits: dict, tracks: dict, offsets: torch.Tensor, n_pixels: int, params=None, states=None,
        stream=None) -> dict:
    E = offsets.numel() - 1
    params = params if params is not None else default_params()
    states = states if states is not None else alloc_states(n_pixels, offsets.device)
    hs, ts, ss = _hits_struct(hits), _tracks_struct(tracks), _states_struct(states)
    _check(lib().velo_fit(C.byref(hs), C.byref(ts), _ptr(offsets), E, int(n_pixels), _geom(),
                          C.byref(params), C.byref(ss), _stream(stream)))
    return states


def fit_momentum(hits: dict, tracks: dict, offsets: torch.Tensor, n_pixels: int, p_mev: torch.Tensor,
                 params=None, states=None, stream=None) -> dict:
    """velo_fit_momentum: the fit with a measured momentum per track slot
    (p_mev: float32 device tensor of at least the track capacity)."""
    E = offsets.numel() - 1
    if p_mev.dtype != torch.float32 or p_mev.numel() < track_capacity(n_pixels):
        raise VeloError("p_mev must be float32 with one value per track slot")
    params = params if params is not None else default_params()
    states = states if states is not None else alloc_states(n_pixels, offsets.device)
    hs, ts, ss = _hits_struct(hits), _tracks_struct(tracks), _states_struct(states)
    _check(lib().velo_fit_momentum(C.byref(hs), C.byref(ts), _ptr(offsets), E, int(n_pixels), _geom(),
                                   C.byref(params), _ptr(p_mev), C.byref(ss), _stream(stream)))
    return states


def reconstruct(pixels: torch.Tensor, offsets: torch.Tensor, params=None, bufs=None, stream=None) -> dict:
    """velo_reconstruct over a packed batch; returns dict(hits, tracks, states, ws)."""
    E = offsets.numel() - 1
    N = _n_pixels(pixels)
    dev = pixels.device
    params = params if params is not None else default_params()
    if bufs is None:
        bufs = dict(hits=alloc_hits(N, E, dev), tracks=alloc_tracks(N, E, dev),
                    states=alloc_states(N, dev), ws=alloc_workspace(N, E, dev))
    hs = _hits_struct(bufs["hits"])
    ts = _tracks_struct(bufs["tracks"])
    ss = _states_struct(bufs["states"])
    ws = bufs["ws"]
    _check(lib().velo_reconstruct(_ptr(pixels), _ptr(offsets), E, N, _geom(), C.byref(params), C.byref(hs),
                                  C.byref(ts), C.byref(ss), _ptr(ws), ws.numel(), _stream(stream)))
    return bufs


# ---------------------------------------------------------------------------
# primary vertices

MAX_PVS = 64
EV_PV_OVERFLOW = 64


class PvParams(C.Structure):
    _fields_ = [("z0", C.c_float), ("bin_w", C.c_float), ("n_bins", C.c_int32), ("max_var", C.c_float),
                ("seed_min", C.c_int32), ("nms", C.c_int32), ("chi2_cut", C.c_float),
                ("n_iter", C.c_int32), ("min_weight", C.c_float)]


class _Pvs(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("n_pv", "z", "var", "weight", "status")]


def default_pv_params(**overrides) -> PvParams:
    p = PvParams()
    lib().velo_pv_params_default(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def alloc_pvs(n_events: int, device="cuda") -> dict:
    E = max(int(n_events), 1)
    f = lambda n, dt=torch.float32: torch.empty(n, dtype=dt, device=device)  # noqa: E731
    return dict(n_pv=f(E, torch.int32), z=f(E * MAX_PVS), var=f(E * MAX_PVS), weight=f(E * MAX_PVS),
                status=f(E, torch.int32))


def find_pvs(tracks: dict, states: dict, offsets, n_pixels: int, params=None, out=None, stream=None):
    """velo_find_pvs: primary vertices from the fitted states of the tracks."""
    E = offsets.numel() - 1
    params = params if params is not None else default_pv_params()
    out = out if out is not None else alloc_pvs(E, offsets.device)
    ts, ss = _tracks_struct(tracks), _states_struct(states)
    ps = _Pvs(*[_ptr(out[k]) for k, _ in _Pvs._fields_])
    _check(lib().velo_find_pvs(C.byref(ts), C.byref(ss), _ptr(offsets), E, int(n_pixels), C.byref(params),
                               C.byref(ps), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# Velo-to-UT search windows

UT_REGIONS = 56
EV_UT_OVERFLOW = 256


class UtParams(C.Structure):
    _fields_ = [("p_min_mev", C.c_float), ("kick_mev", C.c_float), ("z_kick", C.c_float),
                ("tol_u", C.c_float), ("tol_y", C.c_float)]


class _UtOut(C.Structure):
    _fields_ = [(k, C.c_void_p) for k in ("sorted", "region", "status", "win")]


def default_ut_params(**overrides) -> UtParams:
    p = UtParams()
    lib().velo_ut_params_default(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def alloc_ut(n_ut: int, n_events: int, n_pixels: int, device="cuda") -> dict:
    i = lambda n: torch.zeros(max(int(n), 1), dtype=torch.int32, device=device)  # noqa: E731
    return dict(sorted=i(n_ut), region=i(n_events * (UT_REGIONS + 1)), status=i(n_events),
                win=i(track_capacity(n_pixels) * 8))


def ut_windows(ut_words, ut_offsets, tracks: dict, states: dict, offsets, n_pixels: int, params=None,
               out=None, stream=None) -> dict:
    """velo_ut_windows: UT hits sorted into regions and the search window of
    every track slot on every UT plane."""
    E = ut_offsets.numel() - 1
    params = params if params is not None else default_ut_params()
    out = out if out is not None else alloc_ut(ut_words.numel(), E, n_pixels, ut_offsets.device)
    ts, ss = _tracks_struct(tracks), _states_struct(states)
    us = _UtOut(*[_ptr(out[k]) for k, _ in _UtOut._fields_])
    _check(lib().velo_ut_windows(_ptr(ut_words), _ptr(ut_offsets), E, ut_words.numel(), C.byref(ts), C.byref(ss),
                                 _ptr(offsets), int(n_pixels), C.byref(params), C.byref(us), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# streaming form: host memory in, compact tracks and vertices out

EV_GEC = 128
TRACK_ROW = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("tx", "<f4"), ("ty", "<f4"),
                      ("chi2", "<f4"), ("ndof", "<i4"), ("accepted", "u1"), ("nhits", "u1"),
                      ("pad", "<u2")])


class _PipelineConfig(C.Structure):
    _fields_ = [("n_streams", C.c_int32), ("events_per_batch", C.c_uint32),
                ("words_per_batch", C.c_uint64), ("gec_max_words", C.c_uint32)]


class _PipelineResult(C.Structure):
    _fields_ = [("status", C.c_void_p), ("n_tracks", C.c_void_p), ("first_track", C.c_void_p),
                ("tracks", C.c_void_p), ("track_capacity", C.c_uint64), ("n_pv", C.c_void_p),
                ("pv_z", C.c_void_p), ("pv_var", C.c_void_p)]


class Pipeline:
    """velo_pipeline: host-thread / stream pairs with pinned staging; raw
    events from host memory, compact tracks and vertices back to the host."""

    def __init__(self, n_streams: int, events_per_batch: int, words_per_batch: int, gec_max_words: int = 0,
                 params=None, mlp: "Mlp | None" = None, pv_params=None):
        self._h = C.c_void_p()
        cfg = _PipelineConfig(int(n_streams), int(events_per_batch), int(words_per_batch), int(gec_max_words))
        params = params if params is not None else default_params()
        self._keep = mlp  # the classifier's device tensors must outlive the pipeline
        ms = mlp.struct() if mlp is not None else None
        _check(lib().velo_pipeline_create(C.byref(self._h), C.byref(cfg), _geom(), C.byref(params),
                                          C.byref(ms) if ms is not None else None,
                                          C.byref(pv_params) if pv_params is not None else None))

    def close(self):
        if self._h:
            lib().velo_pipeline_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, pixels: np.ndarray, offsets: np.ndarray, with_pvs: bool = True) -> dict:
        px = np.ascontiguousarray(pixels, np.uint32)
        off = np.ascontiguousarray(offsets, np.uint64)
        E = len(off) - 1
        cap = max(len(px) // 3, 1)
        out = dict(status=np.zeros(E, np.uint32), n_tracks=np.zeros(E, np.uint32),
                   first_track=np.zeros(E, np.uint64), tracks=np.zeros(cap, TRACK_ROW))
        if with_pvs:
            out.update(n_pv=np.zeros(E, np.uint32), pv_z=np.zeros((E, MAX_PVS), np.float32),
                       pv_var=np.zeros((E, MAX_PVS), np.float32))
        a = lambda k: C.c_void_p(out[k].ctypes.data) if k in out else C.c_void_p(0)  # noqa: E731
        res = _PipelineResult(a("status"), a("n_tracks"), a("first_track"), a("tracks"), cap, a("n_pv"),
                              a("pv_z"), a("pv_var"))
        rows = C.c_uint64(0)
        _check(lib().velo_pipeline_run(self._h, C.c_void_p(px.ctypes.data), len(px),
                                       C.c_void_p(off.ctypes.data), E, C.byref(res), C.byref(rows)))
        out["tracks"] = out["tracks"][:rows.value]
        return out


NOALLOC_SCRATCH_BYTES = 512 << 20


def reconstruct_noalloc(pixels, offsets, params=None, bufs=None, stream=None) -> dict:
    """velo_reconstruct_noalloc: velo_reconstruct with the library's own device
    scratch (no workspace argument; the library allocates nothing)."""
    E = offsets.numel() - 1
    N = _n_pixels(pixels)
    dev = pixels.device
    params = params if params is not None else default_params()
    if bufs is None:
        bufs = dict(hits=alloc_hits(N, E, dev), tracks=alloc_tracks(N, E, dev), states=alloc_states(N, dev))
    hs, ts, ss = _hits_struct(bufs["hits"]), _tracks_struct(bufs["tracks"]), _states_struct(bufs["states"])
    _check(lib().velo_reconstruct_noalloc(_ptr(pixels), _ptr(offsets), E, N, _geom(), C.byref(params), C.byref(hs),
                                          C.byref(ts), C.byref(ss), _stream(stream)))
    return bufs


class KernelTimer:
    """HIP events (created through the HIP runtime) around the main kernel of
    each stage of velo_reconstruct_timed; durations in milliseconds."""
    STAGES = ("cluster", "find_tracks", "fit")

    def __init__(self):
        self.hip = C.CDLL("libamdhip64.so")
        self.hip.hipEventCreate.argtypes = [C.c_void_p]
        self.hip.hipEventElapsedTime.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p]
        self.hip.hipEventSynchronize.argtypes = [C.c_void_p]
        self.hip.hipEventDestroy.argtypes = [C.c_void_p]
        self.ev = (C.c_void_p * 6)()
        for i in range(6):
            if self.hip.hipEventCreate(C.byref(self.ev, i * C.sizeof(C.c_void_p))) != 0:
                raise VeloError("hipEventCreate failed")

    def durations(self) -> list:
        if self.hip.hipEventSynchronize(self.ev[5]) != 0:
            raise VeloError("hipEventSynchronize failed")
        out = []
        for k in range(3):
            ms = C.c_float(0)
            if self.hip.hipEventElapsedTime(C.byref(ms), self.ev[2 * k], self.ev[2 * k + 1]) != 0:
                raise VeloError("hipEventElapsedTime failed")
            out.append(ms.value)
        return out

    def close(self):
        for i in range(6):
            if self.ev[i]:
                self.hip.hipEventDestroy(self.ev[i])
                self.ev[i] = None


def reconstruct_timed(pixels, offsets, timer: KernelTimer, params=None, bufs=None, stream=None) -> dict:
    """velo_reconstruct_timed: velo_reconstruct with the timer's events around
    the main kernel of each stage (read them with timer.durations())."""
    E = offsets.numel() - 1
    N = _n_pixels(pixels)
    dev = pixels.device
    params = params if params is not None else default_params()
    if bufs is None:
        bufs = dict(hits=alloc_hits(N, E, dev), tracks=alloc_tracks(N, E, dev),
                    states=alloc_states(N, dev), ws=alloc_workspace(N, E, dev))
    hs, ts, ss = _hits_struct(bufs["hits"]), _tracks_struct(bufs["tracks"]), _states_struct(bufs["states"])
    ws = bufs["ws"]
    _check(lib().velo_reconstruct_timed(_ptr(pixels), _ptr(offsets), E, N, _geom(), C.byref(params), C.byref(hs),
                                        C.byref(ts), C.byref(ss), _ptr(ws), ws.numel(), _stream(stream),
                                        timer.ev))
    return bufs


# ---------------------------------------------------------------------------
# learned track-quality classifier


class Mlp:
    """Device-resident classifier: params [1377], mean [8], std [8] (float32
    tensors on the GPU) and the accept threshold on the logit."""

    def __init__(self, params, mean, std, threshold: float):
        self.params, self.mean, self.std, self.threshold = params, mean, std, float(threshold)

    def struct(self):
        return _Mlp(_ptr(self.params), _ptr(self.mean), _ptr(self.std), C.c_float(self.threshold))


def fit_mlp(hits, tracks, offsets, n_pixels, mlp: Mlp, params=None, states=None, stream=None) -> dict:
    E = offsets.numel() - 1
    params = params if params is not None else default_params()
    states = states if states is not None else alloc_states(n_pixels, offsets.device)
    hs, ts, ss, ms = _hits_struct(hits), _tracks_struct(tracks), _states_struct(states), mlp.struct()
    _check(lib().velo_fit_mlp(C.byref(hs), C.byref(ts), _ptr(offsets), E, int(n_pixels), _geom(),
                              C.byref(params), C.byref(ms), C.byref(ss), _stream(stream)))
    return states


def reconstruct_mlp(pixels, offsets, mlp: Mlp, params=None, bufs=None, stream=None) -> dict:
    E = offsets.numel() - 1
    N = _n_pixels(pixels)
    dev = pixels.device
    params = params if params is not None else default_params()
    if bufs is None:
        bufs = dict(hits=alloc_hits(N, E, dev), tracks=alloc_tracks(N, E, dev),
                    states=alloc_states(N, dev), ws=alloc_workspace(N, E, dev))
    hs, ts, ss = _hits_struct(bufs["hits"]), _tracks_struct(bufs["tracks"]), _states_struct(bufs["states"])
    ms = mlp.struct()
    ws = bufs["ws"]
    _check(lib().velo_reconstruct_mlp(_ptr(pixels), _ptr(offsets), E, N, _geom(), C.byref(params), C.byref(ms),
                                      C.byref(hs), C.byref(ts), C.byref(ss), _ptr(ws), ws.numel(),
                                      _stream(stream)))
    return bufs


def track_features(hits, tracks, states, offsets, n_pixels, out=None, stream=None):
    """Raw features of every track slot: float32 [cap, 8]."""
    E = offsets.numel() - 1
    cap = track_capacity(n_pixels)
    out = out if out is not None else torch.zeros((cap, N_FEATURES), dtype=torch.float32,
                                                  device=offsets.device)
    hs, ts, ss = _hits_struct(hits), _tracks_struct(tracks), _states_struct(states)
    _check(lib().velo_track_features(C.byref(hs), C.byref(ts), C.byref(ss), _ptr(offsets), E,
                                     int(n_pixels), _geom(), _ptr(out), _stream(stream)))
    return out


def mlp_workspace(n: int, device="cuda"):
    return torch.empty(int(lib().velo_mlp_workspace_bytes(int(n))), dtype=torch.uint8, device=device)


def feature_stats(feat, ws=None, stream=None):
    n = feat.shape[0]
    mean = torch.empty(N_FEATURES, dtype=torch.float32, device=feat.device)
    std = torch.empty(N_FEATURES, dtype=torch.float32, device=feat.device)
    ws = ws if ws is not None else mlp_workspace(0, feat.device)
    _check(lib().velo_feature_stats(_ptr(feat), n, _ptr(mean), _ptr(std), _ptr(ws), ws.numel(),
                                    _stream(stream)))
    return mean, std


def mlp_fwd_bwd(params, mean, std, feat, label, n, idx=None, grad=None, loss=None, ws=None, stream=None):
    dev = feat.device
    grad = grad if grad is not None else torch.empty(N_PARAMS, dtype=torch.float32, device=dev)
    loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device=dev)
    ws = ws if ws is not None else mlp_workspace(n, dev)
    _check(lib().velo_mlp_fwd_bwd(_ptr(params), _ptr(mean), _ptr(std), _ptr(feat), _ptr(label),
                                  _ptr(idx), int(n), _ptr(grad), _ptr(loss), _ptr(ws), ws.numel(),
                                  _stream(stream)))
    return grad, loss


def mlp_adam_step(params, m, v, grad, step: int, lr: float, stream=None):
    _check(lib().velo_mlp_adam_step(_ptr(params), _ptr(m), _ptr(v), _ptr(grad), int(step),
                                    C.c_float(lr), _stream(stream)))


def mlp_infer(mlp: Mlp, feat, n=None, out=None, stream=None):
    n = feat.shape[0] if n is None else n
    out = out if out is not None else torch.empty(n, dtype=torch.float32, device=feat.device)
    ms = mlp.struct()
    _check(lib().velo_mlp_infer(C.byref(ms), _ptr(feat), int(n), _ptr(out), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# batched form


class Context:
    """velo_context: autotuned launch shapes and the captured HIP graph of the
    batched form (persistent work-stealing kernels)."""

    def __init__(self, params=None, geometry=None):
        self._h = C.c_void_p()
        self._params = params if params is not None else default_params()
        _check(lib().velo_context_create(C.byref(self._h), _geom(geometry), C.byref(self._params)))

    def close(self):
        if self._h:
            lib().velo_context_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    SOURCES = {0: "untuned", 1: "tuned", 2: "tune cache", 3: "set"}

    def config(self) -> dict:
        out = (C.c_int32 * 13)()
        ms = (C.c_float * 5)()
        _check(lib().velo_context_config(self._h, out, ms))
        return dict(tuned=bool(out[0]), source=self.SOURCES.get(out[0], str(out[0])),
                    cluster_grid=out[1], mid_grid=out[2], find_threads=out[3],
                    find_grid=out[4], fit_threads=out[5], tier_grids=[out[6], out[7], out[8]],
                    route_hits=out[9], fork=bool(out[10]), find_order=bool(out[11]), tiny=bool(out[12]),
                    tuned_ms=[float(v) for v in ms[:3]], per_item_ms=[float(ms[3]), float(ms[4])])

    def set_config(self, cluster_grid=0, mid_grid=512, find_threads=256, find_grid=0, fit_threads=128,
                   tier_grids=(512, 256, 128), route_hits=0, fork=False, find_order=False, tiny=False):
        """velo_context_set_config: fixed launch shapes instead of tuning.
        route_hits: 0 no routing, -1 by the small tier's plane capacity only,
        n > 0 also events above n hits (needs find_grid == 0); find_order:
        the first tier takes the events largest first (needs find_grid == 0); tiny: the tiny tier
        ahead of the small one (needs find_grid == 0, 256 lanes, no routing)."""
        v = (C.c_int32 * 12)(cluster_grid, mid_grid, find_threads, find_grid, fit_threads, *tier_grids,
                             route_hits, int(fork), int(find_order), int(tiny))
        _check(lib().velo_context_set_config(self._h, v))

    def mlp_load(self, blob: bytes):
        """velo_mlp_load: the context's own classifier from a blob (mlp_blob)."""
        b = C.create_string_buffer(bytes(blob), len(blob))
        _check(lib().velo_mlp_load(self._h, b, len(blob)))

    def mlp_save(self) -> bytes:
        b = C.create_string_buffer(MLP_BLOB_BYTES)
        _check(lib().velo_mlp_save(self._h, b, MLP_BLOB_BYTES))
        return b.raw

    def mlp_train_step(self, feat, label, n: int, lr: float, step: int, idx=None, loss=None, stream=None):
        """velo_mlp_train_step: one forward / backward pass and Adam update."""
        _check(lib().velo_mlp_train_step(self._h, _ptr(feat), _ptr(label), _ptr(idx), int(n), C.c_float(lr),
                                         int(step), _ptr(loss), _stream(stream)))

    def reconstruct(self, pixels, offsets, params=None, mlp: Mlp | None = None, bufs=None, stream=None):
        E = offsets.numel() - 1
        N = _n_pixels(pixels)
        dev = pixels.device
        params = params if params is not None else default_params()
        if bufs is None:
            bufs = dict(hits=alloc_hits(N, E, dev), tracks=alloc_tracks(N, E, dev),
                        states=alloc_states(N, dev), ws=alloc_batched_workspace(N, E, dev))
        hs, ts, ss = _hits_struct(bufs["hits"]), _tracks_struct(bufs["tracks"]), _states_struct(bufs["states"])
        ms = mlp.struct() if mlp is not None else None
        ws = bufs["ws"]
        _check(lib().velo_reconstruct_batched(self._h, _ptr(pixels), _ptr(offsets), E, N, C.byref(params),
                                              C.byref(ms) if ms is not None else None, C.byref(hs),
                                              C.byref(ts), C.byref(ss), _ptr(ws), ws.numel(),
                                              _stream(stream)))
        return bufs


MLP_BLOB_MAGIC = 0x504C4D56
MLP_BLOB_BYTES = 16 + 4 * (N_PARAMS + 2 * N_FEATURES + 1)


def mlp_blob(params, mean, std, threshold: float) -> bytes:
    """The classifier blob of velo_mlp_load from host arrays (float32)."""
    head = np.array([MLP_BLOB_MAGIC, 1, N_PARAMS, N_FEATURES], np.uint32).tobytes()
    body = np.concatenate([np.asarray(params, np.float32).ravel(), np.asarray(mean, np.float32).ravel(),
                           np.asarray(std, np.float32).ravel(), np.array([threshold], np.float32)])
    assert body.size == N_PARAMS + 2 * N_FEATURES + 1
    return head + body.astype(np.float32).tobytes()


def parse_mlp_blob(blob: bytes):
    """(params, mean, std, threshold) of a blob."""
    v = np.frombuffer(blob, np.float32, offset=16)
    return v[:N_PARAMS].copy(), v[N_PARAMS:N_PARAMS + 8].copy(), v[N_PARAMS + 8:N_PARAMS + 16].copy(), float(v[-1])


def check_status(status_a, status_b=None, n_events=None, stream=None):
    """velo_check_status: (0 or VELO_ERR_INPUT, OR of the status words)."""
    t = status_a if status_a is not None else status_b
    n = t.numel() if n_events is None else n_events
    word = torch.empty(1, dtype=torch.int32, device=t.device)
    h = C.c_uint32(0)
    rc = lib().velo_check_status(_ptr(status_a), _ptr(status_b), int(n), _ptr(word), C.byref(h), _stream(stream))
    if rc not in (0, 2):
        _check(rc)
    return rc, h.value


def batched_workspace_bytes(n_pixels: int, n_events: int) -> int:
    return int(lib().velo_batched_workspace_bytes(int(n_pixels), int(n_events)))


def alloc_batched_workspace(n_pixels: int, n_events: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(batched_workspace_bytes(n_pixels, n_events), 1), dtype=torch.uint8,
                       device=device)
