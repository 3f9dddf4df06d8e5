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
        L.velo_workspace_bytes.argtypes = [C.c_uint64, C.c_uint32]
        L.velo_workspace_bytes.restype = C.c_size_t
        L.velo_cluster.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, C.c_size_t, P]
        L.velo_cluster.restype = C.c_int
        L.velo_find_tracks.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, P, C.c_size_t, P]
        L.velo_find_tracks.restype = C.c_int
        L.velo_fit.argtypes = [P, P, P, C.c_uint32, C.c_uint64, P, P, P]
        L.velo_fit.restype = C.c_int
        L.velo_reconstruct.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, P, P, P, C.c_size_t, P]
        L.velo_reconstruct.restype = C.c_int
        L.velo_status_string.argtypes = [C.c_int]
        L.velo_status_string.restype = C.c_char_p
        L.velo_fit_mlp.argtypes = [P, P, P, C.c_uint32, C.c_uint64, P, P, P, P]
        L.velo_fit_mlp.restype = C.c_int
        L.velo_reconstruct_mlp.argtypes = [P, P, C.c_uint32, C.c_uint64, P, P, P, P, P, P, C.c_size_t, P]
        L.velo_reconstruct_mlp.restype = C.c_int
        L.velo_track_features.argtypes = [P, P, P, P, C.c_uint32, C.c_uint64, P, P]
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
        L.velo_context_create.argtypes = [P]
        L.velo_context_create.restype = C.c_int
        L.velo_context_destroy.argtypes = [P]
        L.velo_context_destroy.restype = None
        L.velo_context_config.argtypes = [P, P, P]
        L.velo_context_config.restype = C.c_int
        L.velo_batched_workspace_bytes.argtypes = [C.c_uint64, C.c_uint32]
        L.velo_batched_workspace_bytes.restype = C.c_size_t
        L.velo_reconstruct_batched.argtypes = [P, P, P, C.c_uint32, C.c_uint64, P, P, P, P, P, P,
                                               C.c_size_t, P]
        L.velo_reconstruct_batched.restype = C.c_int
        _lib = L
    return _lib


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
    _check(lib().velo_cluster(_ptr(pixels), _ptr(offsets), E, N, C.byref(hs), _ptr(ws),
                              ws.numel(), _stream(stream)))
    return hits


def find_tracks(hits: dict, offsets: torch.Tensor, n_pixels: int, params=None, tracks=None, ws=None,
                stream=None) -> dict:
    E = offsets.numel() - 1
    params = params if params is not None else default_params()
    tracks = tracks if tracks is not None else alloc_tracks(n_pixels, E, offsets.device)
    ws = ws if ws is not None else alloc_workspace(n_pixels, E, offsets.device)
    hs, ts = _hits_struct(hits), _tracks_struct(tracks)
    _check(lib().velo_find_tracks(C.byref(hs), _ptr(offsets), E, int(n_pixels), C.byref(params),
                                  C.byref(ts), _ptr(ws), ws.numel(), _stream(stream)))
    return tracks


def fit(hits: dict, tracks: dict, offsets: torch.Tensor, n_pixels: int, params=None, states=None,
        stream=None) -> dict:
    E = offsets.numel() - 1
    params = params if params is not None else default_params()
    states = states if states is not None else alloc_states(n_pixels, offsets.device)
    hs, ts, ss = _hits_struct(hits), _tracks_struct(tracks), _states_struct(states)
    _check(lib().velo_fit(C.byref(hs), C.byref(ts), _ptr(offsets), E, int(n_pixels),
                          C.byref(params), C.byref(ss), _stream(stream)))
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
    _check(lib().velo_reconstruct(_ptr(pixels), _ptr(offsets), E, N, C.byref(params), C.byref(hs),
                                  C.byref(ts), C.byref(ss), _ptr(ws), ws.numel(), _stream(stream)))
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
    _check(lib().velo_fit_mlp(C.byref(hs), C.byref(ts), _ptr(offsets), E, int(n_pixels),
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
    _check(lib().velo_reconstruct_mlp(_ptr(pixels), _ptr(offsets), E, N, C.byref(params), C.byref(ms),
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
                                     int(n_pixels), _ptr(out), _stream(stream)))
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

    def __init__(self):
        self._h = C.c_void_p()
        _check(lib().velo_context_create(C.byref(self._h)))

    def close(self):
        if self._h:
            lib().velo_context_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def config(self) -> dict:
        out = (C.c_int32 * 6)()
        ms = (C.c_float * 5)()
        _check(lib().velo_context_config(self._h, out, ms))
        return dict(tuned=bool(out[0]), cluster_grid=out[1], mid_grid=out[2], find_threads=out[3],
                    find_grid=out[4], fit_threads=out[5], tuned_ms=[float(v) for v in ms[:3]],
                    per_item_ms=[float(ms[3]), float(ms[4])])

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


def batched_workspace_bytes(n_pixels: int, n_events: int) -> int:
    return int(lib().velo_batched_workspace_bytes(int(n_pixels), int(n_events)))


def alloc_batched_workspace(n_pixels: int, n_events: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(batched_workspace_bytes(n_pixels, n_events), 1), dtype=torch.uint8,
                       device=device)
