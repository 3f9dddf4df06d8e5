"""The C ABI: libvelo.so loads and exports every function include/velo.h
declares; host-side argument checks reject bad calls before any launch."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "velo.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(velo_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for n in ("velo_cluster", "velo_find_tracks", "velo_fit", "velo_reconstruct",
              "velo_workspace_bytes", "velo_params_default", "velo_status_string"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1912_09161_amd as velo
    L = velo.lib()
    for n in declared_functions():
        assert hasattr(L, n), n


def test_host_argument_checks():
    import paper_1912_09161_amd as velo
    L = velo.lib()
    p = velo.default_params()
    assert abs(p.pt0_mev - 400.0) < 1e-6 and p.max_skip == 1
    # zero events: nothing to do
    g = velo.default_geometry()
    G = C.byref(g)
    assert L.velo_cluster(None, None, 0, 0, G, None, None, 0, None) == 0
    # null buffers are rejected before anything is enqueued
    assert L.velo_cluster(None, None, 3, 10, G, None, None, 0, None) == 1
    assert L.velo_find_tracks(None, None, 3, 10, G, C.byref(p), None, None, 0, None) == 1
    assert L.velo_fit(None, None, None, 3, 10, G, C.byref(p), None, None) == 1
    assert L.velo_status_string(1) == b"invalid argument"
    assert L.velo_workspace_bytes(1000, 10) >= L.velo_workspace_bytes(10, 10) > 0


def test_workspace_too_small_is_reported():
    import paper_1912_09161_amd as velo
    L = velo.lib()
    fake = C.c_void_p(0x1000)
    hits = velo.velo._Hits(*[fake] * 8)
    rc = L.velo_cluster(fake, fake, 2, 100, C.byref(velo.default_geometry()), C.byref(hits), fake, 16, None)
    assert rc == 3


def test_noalloc_rejects_batches_beyond_its_scratch():
    """velo_reconstruct_noalloc refuses a batch whose workspace exceeds its
    device array before touching the GPU (no HIP call is made)."""
    import paper_1912_09161_amd as velo
    L = velo.lib()
    fake = C.c_void_p(0x1000)
    p = velo.default_params()
    hits = velo.velo._Hits(*[fake] * 8)
    tracks = velo.velo._Tracks(*[fake] * 4)
    states = velo.velo._States(*[fake] * 11)
    n_px, n_ev = 10 ** 8, 20000
    assert L.velo_workspace_bytes(n_px, n_ev) > velo.NOALLOC_SCRATCH_BYTES
    G = C.byref(velo.default_geometry())
    rc = L.velo_reconstruct_noalloc(fake, fake, n_ev, n_px, G, C.byref(p), C.byref(hits), C.byref(tracks),
                                    C.byref(states), None)
    assert rc == 3
    assert L.velo_reconstruct_noalloc(None, None, 0, 0, G, C.byref(p), None, None, None, None) == 0
    assert L.velo_reconstruct_noalloc(fake, None, 3, 10, G, C.byref(p), C.byref(hits), C.byref(tracks),
                                      C.byref(states), None) == 1


def test_mlp_blob_is_checked_before_any_device_use():
    """velo_mlp_load rejects a blob of the wrong size, magic, version, shape,
    a non-finite value or a non-positive standard deviation, leaving the
    context without a classifier (no device call is made)."""
    import numpy as np

    import paper_1912_09161_amd as velo
    L = velo.lib()
    ctx = velo.Context()
    good = velo.mlp_blob(np.zeros(1377), np.zeros(8), np.ones(8), 0.5)
    assert len(good) == velo.velo.MLP_BLOB_BYTES
    p, m, s, t = velo.parse_mlp_blob(good)
    assert t == 0.5 and (s == 1).all()
    bad = [good[:-4], b"XXXX" + good[4:],
           good[:4] + np.uint32(2).tobytes() + good[8:],
           good[:8] + np.uint32(1376).tobytes() + good[12:],
           velo.mlp_blob(np.full(1377, np.nan), np.zeros(8), np.ones(8), 0.5),
           velo.mlp_blob(np.zeros(1377), np.zeros(8), np.zeros(8), 0.5),
           velo.mlp_blob(np.zeros(1377), np.zeros(8), np.ones(8), np.inf)]
    for b in bad:
        buf = C.create_string_buffer(b, len(b))
        assert L.velo_mlp_load(ctx._h, buf, len(b)) == 1
    out = C.create_string_buffer(len(good))
    assert L.velo_mlp_save(ctx._h, out, len(good)) == 1  # nothing loaded
    assert L.velo_mlp_train_step(ctx._h, None, None, None, 10, C.c_float(1e-3), 1, None, None) == 1
    ctx.close()


def test_check_status_arguments():
    import paper_1912_09161_amd as velo
    L = velo.lib()
    h = C.c_uint32(7)
    assert L.velo_check_status(None, None, 5, C.c_void_p(0x1000), C.byref(h), None) == 1
    assert L.velo_check_status(C.c_void_p(0x1000), None, 0, C.c_void_p(0x1000), C.byref(h), None) == 0
    assert h.value == 0
    assert L.velo_status_string(2) == b"at least one event is flagged"


def test_geometry_is_checked():
    """The built-in detector model is accepted; any other statement of it (a
    plane moved by one ulp, another pitch, sensor size or hole, a missing
    geometry) is rejected before anything is enqueued, by every call that
    takes one."""
    import numpy as np

    import paper_1912_09161_amd as velo
    L = velo.lib()
    g = velo.default_geometry()
    assert g.n_layers == 26 and g.n_cols == 1536 and abs(g.pitch_mm - 0.055) < 1e-7
    assert g.z_mm[0] == np.float32(-280.0) and g.z_mm[25] == np.float32(750.0)
    assert g.z_mm[1] == np.float32(-280.0 + 1030.0 / 25.0)
    fake = C.c_void_p(0x1000)
    hits = velo.velo._Hits(*[fake] * 8)
    p = velo.default_params()
    ok = L.velo_cluster(fake, fake, 2, 100, C.byref(g), C.byref(hits), fake, 16, None)
    assert ok == 3  # passes the geometry check, fails on the workspace size

    def variants():
        for f, v in (("pitch_mm", 0.05), ("n_cols", 1024), ("n_rows", 1535), ("hole_r_mm", 5.0),
                     ("n_layers", 25)):
            b = velo.default_geometry()
            setattr(b, f, v)
            yield b
        b = velo.default_geometry()
        b.z_mm[7] = float(np.nextafter(np.float32(b.z_mm[7]), np.float32(1e9)))
        yield b

    for b in variants():
        assert L.velo_cluster(fake, fake, 2, 100, C.byref(b), C.byref(hits), fake, 16, None) == 1
        assert L.velo_find_tracks(C.byref(hits), fake, 2, 100, C.byref(b), C.byref(p), fake, fake, 16,
                                  None) == 1
        ctx = C.c_void_p()
        assert L.velo_context_create(C.byref(ctx), C.byref(b), C.byref(p)) == 1
    assert L.velo_cluster(fake, fake, 2, 100, None, C.byref(hits), fake, 16, None) == 1


def test_context_shapes_are_checked_on_the_host():
    """velo_context_set_config checks every field and their combinations
    (routing, fork, event order and the tiny tier need one workgroup per
    event; the fork needs routing; the tiny tier needs 256 lanes and no
    routing) before touching the context, and velo_context_config reports
    what was set.  No device call is made."""
    import paper_1912_09161_amd as velo
    base = dict(cluster_grid=0, mid_grid=512, find_threads=256, find_grid=0, fit_threads=128,
                tier_grids=(512, 256, 128))
    good = [dict(base), dict(base, cluster_grid=2048, find_grid=1024, tier_grids=(16, 8, 8)),
            dict(base, route_hits=-1, fork=True, find_order=True), dict(base, route_hits=3000),
            dict(base, tiny=True, find_order=True), dict(base, find_threads=128, route_hits=1)]
    bad = [dict(find_threads=192), dict(fit_threads=32), dict(mid_grid=0), dict(cluster_grid=-1),
           dict(find_grid=70000), dict(tier_grids=(0, 8, 8)), dict(tier_grids=(513, 8, 8)),
           dict(route_hits=-2), dict(route_hits=5, find_grid=512), dict(fork=True),
           dict(find_order=True, find_grid=512), dict(tiny=True, find_grid=512),
           dict(tiny=True, route_hits=-1), dict(tiny=True, find_threads=128)]
    ctx = velo.Context()
    assert ctx.config()["source"] == "untuned"
    for b in bad:
        with pytest.raises(velo.VeloError):
            ctx.set_config(**dict(base, **b))
        assert ctx.config()["source"] == "untuned"
    for g in good:
        ctx.set_config(**g)
        cfg = ctx.config()
        assert cfg["source"] == "set"
        for k, v in g.items():
            assert cfg[k] == (list(v) if isinstance(v, tuple) else v), (k, cfg[k], v)
    ctx.close()
