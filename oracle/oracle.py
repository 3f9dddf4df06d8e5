"""ctypes binding of the C oracle (test infrastructure only).

Array conventions follow `velo_oracle.h`: hits live at absolute slot
offsets[e] + layer_start[e, l] + rank, tracks at floor(offsets[e] / 3) + t.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRCS = [os.path.join(_HERE, f) for f in ("velo_oracle.c", "velo_oracle_mlp.c", "velo_oracle_pv.c",
                                          "velo_oracle_ut.c")]
_LIB = os.path.join(_HERE, "libvelo_oracle.so")

EV_BAD_WORD = 1
EV_LAYER_ORDER = 2
EV_DUPLICATE = 4
EV_HOLE = 8
EV_OVERFLOW = 16
EV_BAD_OFFSETS = 32
EV_PV_OVERFLOW = 64
EV_UT_OVERFLOW = 256
UT_SECTORS = 14
UT_REGIONS = 56
UT_MAX_HITS = 8192
MAX_CANDIDATES = 65536
MAX_PVS = 64

# Default cut and filter constants (a reading of the paper, which gives only
# the 400 MeV transverse momentum of the scattering model).
DEFAULT_PARAMS = dict(
    max_t=0.4, sin2_phi=9e-4, s_seed=0.025, s_fwd=0.04, max_skip=1,
    sigma_meas=0.055 / 12 ** 0.5, pt0_mev=400.0, x_over_x0=5.94e-4, qc3=4.0, qc4=10.0,
)


class _Params(C.Structure):
    _fields_ = [("max_t", C.c_float), ("sin2_phi", C.c_float), ("s_seed", C.c_float),
                ("s_fwd", C.c_float), ("max_skip", C.c_int32), ("sigma_meas", C.c_float),
                ("pt0_mev", C.c_float), ("x_over_x0", C.c_float), ("qc3", C.c_float),
                ("qc4", C.c_float)]


def lib_path() -> str:
    return _LIB


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no contraction, no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-ffp-contract=off",
                               "-fno-fast-math", "-shared", "-fPIC", *_SRCS, "-lm", "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _L():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = C.CDLL(_LIB)
        P = C.c_void_p
        lib.velo_oracle_cluster.restype = C.c_uint32
        lib.velo_oracle_cluster.argtypes = [P, P, C.c_uint32, C.c_uint32, C.c_uint64] + [P] * 8
        lib.velo_oracle_find_tracks.restype = None
        lib.velo_oracle_find_tracks.argtypes = [P, P, P, P, P, P, C.c_uint32, P, P, P, P, P]
        lib.velo_oracle_fit.restype = None
        lib.velo_oracle_fit.argtypes = [P, P, P, P, C.c_uint32, P, P, P, P] + [P] * 10
        lib.velo_oracle_fit_momentum.restype = None
        lib.velo_oracle_fit_momentum.argtypes = [P, P, P, P, C.c_uint32, P, P, P, P, P] + [P] * 10
        lib.velo_oracle_fit_points_p.restype = C.c_int32
        lib.velo_oracle_fit_points_p.argtypes = [P, P, P, P, C.c_int32, C.c_float, P, P, P, P, P]
        lib.velo_oracle_fit_points.restype = C.c_int32
        lib.velo_oracle_fit_points.argtypes = [P, P, P, P, C.c_int32, P, P, P, P, P]
        lib.velo_oracle_layer_z.restype = C.c_float
        lib.velo_oracle_layer_z.argtypes = [C.c_int32]
        lib.velo_oracle_mlp_nparams.restype = C.c_int32
        lib.velo_oracle_features.restype = None
        lib.velo_oracle_features.argtypes = [P, P, C.c_uint32, P, P, P, P, P, P, P, P]
        lib.velo_oracle_mlp_fwd_bwd.restype = C.c_double
        lib.velo_oracle_mlp_fwd_bwd.argtypes = [P, P, P, C.c_int64, P]
        lib.velo_oracle_mlp_forward.restype = None
        lib.velo_oracle_mlp_forward.argtypes = [P, P, C.c_int64, P]
        lib.velo_oracle_pv_params_default.restype = None
        lib.velo_oracle_pv_params_default.argtypes = [P]
        lib.velo_oracle_find_pvs.restype = None
        lib.velo_oracle_find_pvs.argtypes = [P, C.c_uint32] + [P] * 13
        lib.velo_oracle_ut_params_default.restype = None
        lib.velo_oracle_ut_params_default.argtypes = [P]
        lib.velo_oracle_ut_strip_u.restype = C.c_float
        lib.velo_oracle_ut_strip_u.argtypes = [C.c_uint32]
        lib.velo_oracle_ut.restype = None
        lib.velo_oracle_ut.argtypes = [P, P, C.c_uint32, C.c_uint64, P, C.c_uint64] + [P] * 12
        lib.velo_oracle_mlp_forward_bf16.restype = None
        lib.velo_oracle_mlp_forward_bf16.argtypes = [P, P, P, P, C.c_int64, P]
        _lib = lib
    return _lib


def _p(a: np.ndarray, off: int = 0):
    return C.c_void_p(a.ctypes.data + off * a.itemsize)


def _params(params) -> _Params:
    d = dict(DEFAULT_PARAMS)
    if params:
        d.update(params)
    return _Params(**{k: d[k] for k, _ in _Params._fields_})


def layer_z(l: int) -> float:
    return float(_L().velo_oracle_layer_z(int(l)))


def cluster(pixels, offsets, events=None) -> dict:
    """Cluster all events (or the half-open event range `events`); the batch
    holds len(pixels) words."""
    pixels = np.ascontiguousarray(pixels, np.uint32)
    offsets = np.ascontiguousarray(offsets, np.uint64)
    E = len(offsets) - 1
    e0, e1 = (0, E) if events is None else events
    N = max(len(pixels), 1)
    out = dict(x=np.zeros(N, np.float32), y=np.zeros(N, np.float32),
               key=np.zeros(N, np.uint32), aux=np.zeros(N, np.uint32),
               layer_start=np.zeros((E, 27), np.uint32), layer_nhits=np.zeros((E, 26), np.uint32),
               n_hits=np.zeros(E, np.uint32), status=np.zeros(E, np.uint32))
    cluster_into(pixels, offsets, e0, e1, out)
    return out


def cluster_into(pixels, offsets, e0, e1, out):
    if e1 <= e0:
        return
    _L().velo_oracle_cluster(_p(pixels), _p(offsets), e0, e1, len(pixels),
                             _p(out["x"]), _p(out["y"]), _p(out["key"]), _p(out["aux"]),
                             _p(out["layer_start"]), _p(out["layer_nhits"]),
                             _p(out["n_hits"]), _p(out["status"]))


def find_tracks(hits: dict, offsets, params=None, events=None) -> dict:
    offsets = np.ascontiguousarray(offsets, np.uint64)
    E = len(offsets) - 1
    e0, e1 = (0, E) if events is None else events
    cap = max(len(hits["x"]) // 3, 1)
    out = dict(n_tracks=np.zeros(E, np.uint32), nhits=np.zeros(cap, np.uint8),
               hit_idx=np.zeros((cap, 26), np.uint32), status=np.zeros(E, np.uint32))
    find_into(hits, offsets, e0, e1, _params(params), out)
    return out


def find_into(hits, offsets, e0, e1, P, out):
    if e1 <= e0:
        return
    _L().velo_oracle_find_tracks(_p(hits["x"]), _p(hits["y"]), _p(hits["key"]),
                                 _p(hits["layer_start"], 27 * e0), _p(hits["layer_nhits"], 26 * e0),
                                 _p(offsets, e0), e1 - e0, C.byref(P),
                                 _p(out["n_tracks"], e0), _p(out["nhits"]), _p(out["hit_idx"]),
                                 _p(out["status"], e0))


def fit(hits: dict, tracks: dict, offsets, params=None, events=None) -> dict:
    offsets = np.ascontiguousarray(offsets, np.uint64)
    E = len(offsets) - 1
    e0, e1 = (0, E) if events is None else events
    cap = max(len(hits["x"]) // 3, 1)
    f = lambda: np.zeros(cap, np.float32)  # noqa: E731
    out = dict(x=f(), y=f(), z=f(), tx=f(), ty=f(), cov_x=np.zeros((cap, 3), np.float32),
               cov_y=np.zeros((cap, 3), np.float32), chi2=f(), ndof=np.zeros(cap, np.int32),
               accepted=np.zeros(cap, np.uint8))
    fit_into(hits, tracks, offsets, e0, e1, _params(params), out)
    return out


def fit_into(hits, tracks, offsets, e0, e1, P, out):
    if e1 <= e0:
        return
    _L().velo_oracle_fit(_p(hits["x"]), _p(hits["y"]), _p(hits["key"]), _p(offsets, e0), e1 - e0,
                         _p(tracks["n_tracks"], e0), _p(tracks["nhits"]), _p(tracks["hit_idx"]),
                         C.byref(P), _p(out["x"]), _p(out["y"]), _p(out["z"]), _p(out["tx"]),
                         _p(out["ty"]), _p(out["cov_x"]), _p(out["cov_y"]), _p(out["chi2"]),
                         _p(out["ndof"]), _p(out["accepted"]))


def fit_momentum(hits: dict, tracks: dict, offsets, p_mev, params=None) -> dict:
    """The fit with a measured momentum per track slot (velo_oracle_fit_momentum)."""
    offsets = np.ascontiguousarray(offsets, np.uint64)
    E = len(offsets) - 1
    cap = max(len(hits["x"]) // 3, 1)
    pm = np.zeros(cap, np.float32)
    pm[:len(p_mev)] = np.asarray(p_mev, np.float32)[:cap]
    f = lambda: np.zeros(cap, np.float32)  # noqa: E731
    out = dict(x=f(), y=f(), z=f(), tx=f(), ty=f(), cov_x=np.zeros((cap, 3), np.float32),
               cov_y=np.zeros((cap, 3), np.float32), chi2=f(), ndof=np.zeros(cap, np.int32),
               accepted=np.zeros(cap, np.uint8))
    P = _params(params)
    _L().velo_oracle_fit_momentum(_p(hits["x"]), _p(hits["y"]), _p(hits["key"]), _p(offsets), E,
                                  _p(tracks["n_tracks"]), _p(tracks["nhits"]), _p(tracks["hit_idx"]),
                                  _p(pm), C.byref(P), _p(out["x"]), _p(out["y"]), _p(out["z"]),
                                  _p(out["tx"]), _p(out["ty"]), _p(out["cov_x"]), _p(out["cov_y"]),
                                  _p(out["chi2"]), _p(out["ndof"]), _p(out["accepted"]))
    return out


def fit_points_p(hx, hy, hz, hlayer, p_mev, params=None):
    """Fit one track from explicit hit coordinates with a measured momentum."""
    hx = np.ascontiguousarray(hx, np.float32)
    hy = np.ascontiguousarray(hy, np.float32)
    hz = np.ascontiguousarray(hz, np.float32)
    hl = np.ascontiguousarray(hlayer, np.int32)
    o5 = np.zeros(5, np.float32)
    cx = np.zeros(3, np.float32)
    cy = np.zeros(3, np.float32)
    chi2 = np.zeros(1, np.float32)
    P = _params(params)
    nd = _L().velo_oracle_fit_points_p(_p(hx), _p(hy), _p(hz), _p(hl), len(hx), C.c_float(p_mev),
                                       C.byref(P), _p(o5), _p(cx), _p(cy), _p(chi2))
    return dict(x=o5[0], y=o5[1], z=o5[2], tx=o5[3], ty=o5[4], cov_x=cx, cov_y=cy,
                chi2=float(chi2[0]), ndof=int(nd))


def fit_points(hx, hy, hz, hlayer, params=None):
    """Fit one track from explicit hit coordinates (decreasing z)."""
    hx = np.ascontiguousarray(hx, np.float32)
    hy = np.ascontiguousarray(hy, np.float32)
    hz = np.ascontiguousarray(hz, np.float32)
    hl = np.ascontiguousarray(hlayer, np.int32)
    o5 = np.zeros(5, np.float32)
    cx = np.zeros(3, np.float32)
    cy = np.zeros(3, np.float32)
    chi2 = np.zeros(1, np.float32)
    P = _params(params)
    nd = _L().velo_oracle_fit_points(_p(hx), _p(hy), _p(hz), _p(hl), len(hx), C.byref(P),
                                     _p(o5), _p(cx), _p(cy), _p(chi2))
    return dict(x=o5[0], y=o5[1], z=o5[2], tx=o5[3], ty=o5[4], cov_x=cx, cov_y=cy,
                chi2=float(chi2[0]), ndof=int(nd))


def reconstruct(pixels, offsets, params=None, events=None, threads: int = 1) -> dict:
    """cluster -> find -> fit on a thread pool over contiguous event ranges
    (the batch holds len(pixels) words)."""
    pixels = np.ascontiguousarray(pixels, np.uint32)
    offsets = np.ascontiguousarray(offsets, np.uint64)
    E = len(offsets) - 1
    e0, e1 = (0, E) if events is None else events
    N = max(len(pixels), 1)
    cap = max(len(pixels) // 3, 1)
    P = _params(params)
    hits = dict(x=np.zeros(N, np.float32), y=np.zeros(N, np.float32),
                key=np.zeros(N, np.uint32), aux=np.zeros(N, np.uint32),
                layer_start=np.zeros((E, 27), np.uint32), layer_nhits=np.zeros((E, 26), np.uint32),
                n_hits=np.zeros(E, np.uint32), status=np.zeros(E, np.uint32))
    tracks = dict(n_tracks=np.zeros(E, np.uint32), nhits=np.zeros(cap, np.uint8),
                  hit_idx=np.zeros((cap, 26), np.uint32), status=np.zeros(E, np.uint32))
    f = lambda: np.zeros(cap, np.float32)  # noqa: E731
    states = dict(x=f(), y=f(), z=f(), tx=f(), ty=f(), cov_x=np.zeros((cap, 3), np.float32),
                  cov_y=np.zeros((cap, 3), np.float32), chi2=f(), ndof=np.zeros(cap, np.int32),
                  accepted=np.zeros(cap, np.uint8))

    def run(a, b):
        cluster_into(pixels, offsets, a, b, hits)
        find_into(hits, offsets, a, b, P, tracks)
        fit_into(hits, tracks, offsets, a, b, P, states)

    if threads <= 1 or e1 - e0 < 2:
        run(e0, e1)
    else:
        from concurrent.futures import ThreadPoolExecutor
        step = max(1, (e1 - e0 + 4 * threads - 1) // (4 * threads))
        ranges = [(a, min(a + step, e1)) for a in range(e0, e1, step)]
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(lambda r: run(*r), ranges))
    return dict(hits=hits, tracks=tracks, states=states)


# ---------------------------------------------------------------------------
# learned track-quality classifier

N_FEATURES = 8
N_PARAMS = 1377


def features(hits, tracks, states, offsets) -> np.ndarray:
    """Raw features (double) of every track slot, shape (cap, 8)."""
    offsets = np.ascontiguousarray(offsets, np.uint64)
    E = len(offsets) - 1
    cap = len(tracks["nhits"])
    out = np.zeros((cap, 8), np.float64)
    key = np.ascontiguousarray(hits["key"], np.uint32)
    nt = np.ascontiguousarray(tracks["n_tracks"], np.uint32)
    nh = np.ascontiguousarray(tracks["nhits"], np.uint8)
    hi = np.ascontiguousarray(tracks["hit_idx"], np.uint32)
    tx = np.ascontiguousarray(states["tx"], np.float32)
    ty = np.ascontiguousarray(states["ty"], np.float32)
    ch = np.ascontiguousarray(states["chi2"], np.float32)
    nd = np.ascontiguousarray(states["ndof"], np.int32)
    _L().velo_oracle_features(_p(key), _p(offsets), E, _p(nt), _p(nh), _p(hi), _p(tx), _p(ty),
                              _p(ch), _p(nd), _p(out))
    return out


def mlp_fwd_bwd(params, g, y):
    """(mean loss, gradient) in double over standardised samples g (n, 8)."""
    p = np.ascontiguousarray(params, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    grad = np.zeros(N_PARAMS, np.float64)
    loss = _L().velo_oracle_mlp_fwd_bwd(_p(p), _p(g), _p(y), len(y), _p(grad))
    return float(loss), grad


def mlp_forward(params, g):
    p = np.ascontiguousarray(params, np.float64)
    g = np.ascontiguousarray(g, np.float64)
    z = np.zeros(len(g), np.float64)
    _L().velo_oracle_mlp_forward(_p(p), _p(g), len(g), _p(z))
    return z


def mlp_forward_bf16(params, mean, std, f):
    """Logits in the GPU inference precision from raw binary32 features f (n, 8)."""
    p = np.ascontiguousarray(params, np.float32)
    m = np.ascontiguousarray(mean, np.float32)
    s = np.ascontiguousarray(std, np.float32)
    f = np.ascontiguousarray(f, np.float32)
    z = np.zeros(len(f), np.float32)
    _L().velo_oracle_mlp_forward_bf16(_p(p), _p(m), _p(s), _p(f), len(f), _p(z))
    return z


# ---------------------------------------------------------------------------
# primary vertices


class PvParams(C.Structure):
    _fields_ = [("z0", C.c_float), ("bin_w", C.c_float), ("n_bins", C.c_int32), ("max_var", C.c_float),
                ("seed_min", C.c_int32), ("nms", C.c_int32), ("chi2_cut", C.c_float),
                ("n_iter", C.c_int32), ("min_weight", C.c_float)]


def pv_params(**overrides) -> PvParams:
    p = PvParams()
    _L().velo_oracle_pv_params_default(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def find_pvs(states: dict, tracks: dict, offsets, params: PvParams | None = None) -> dict:
    """PVs of every event from fitted states (velo_oracle_find_pvs)."""
    offsets = np.ascontiguousarray(offsets, np.uint64)
    E = len(offsets) - 1
    P = params if params is not None else pv_params()
    f32 = lambda k: np.ascontiguousarray(states[k], np.float32).ravel()  # noqa: E731
    nt = np.ascontiguousarray(tracks["n_tracks"], np.uint32)
    acc = np.ascontiguousarray(states["accepted"], np.uint8)
    out = dict(n_pv=np.zeros(E, np.uint32), z=np.zeros((E, MAX_PVS), np.float32),
               var=np.zeros((E, MAX_PVS), np.float32), weight=np.zeros((E, MAX_PVS), np.float32),
               status=np.zeros(E, np.uint32))
    z, tx, ty, cx, cy = f32("z"), f32("tx"), f32("ty"), f32("cov_x"), f32("cov_y")
    _L().velo_oracle_find_pvs(_p(offsets), E, _p(nt), _p(z), _p(tx), _p(ty), _p(cx), _p(cy), _p(acc),
                              C.byref(P), _p(out["n_pv"]), _p(out["z"]), _p(out["var"]),
                              _p(out["weight"]), _p(out["status"]))
    return out


class UtParams(C.Structure):
    _fields_ = [("p_min_mev", C.c_float), ("kick_mev", C.c_float), ("z_kick", C.c_float),
                ("tol_u", C.c_float), ("tol_y", C.c_float)]


def ut_params(**overrides) -> UtParams:
    p = UtParams()
    _L().velo_oracle_ut_params_default(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def ut_strip_u(strip: int) -> float:
    """u of a strip's centre (binary32), mm."""
    return float(_L().velo_oracle_ut_strip_u(int(strip)))


def ut_windows(ut_words, ut_offsets, offsets, tracks: dict, states: dict, params: UtParams | None = None,
               n_pixels: int | None = None) -> dict:
    """UT hits sorted into regions and the windows of every track slot
    (velo_oracle_ut): sorted[M], region[E, 57], status[E], win[cap, 8].
    n_pixels defaults to offsets[-1]."""
    w = np.ascontiguousarray(ut_words, np.uint32)
    uo = np.ascontiguousarray(ut_offsets, np.uint64)
    offsets = np.ascontiguousarray(offsets, np.uint64)
    E = len(uo) - 1
    P = params if params is not None else ut_params()
    f32 = lambda k: np.ascontiguousarray(states[k], np.float32).ravel()  # noqa: E731
    nt = np.ascontiguousarray(tracks["n_tracks"], np.uint32)
    acc = np.ascontiguousarray(states["accepted"], np.uint8)
    cap = len(acc)
    out = dict(sorted=np.zeros(max(len(w), 1), np.uint32), region=np.zeros((E, 57), np.uint32),
               status=np.zeros(E, np.uint32), win=np.zeros((cap, 8), np.uint32))
    x, y, z, tx, ty = f32("x"), f32("y"), f32("z"), f32("tx"), f32("ty")
    npx = int(offsets[-1]) if n_pixels is None else int(n_pixels)
    _L().velo_oracle_ut(_p(w), _p(uo), E, len(w), _p(offsets), npx, _p(nt), _p(x), _p(y), _p(z), _p(tx), _p(ty),
                        _p(acc), C.byref(P), _p(out["sorted"]), _p(out["region"]), _p(out["status"]),
                        _p(out["win"]))
    return out
