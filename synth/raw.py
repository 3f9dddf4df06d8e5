"""Hand-built raw events for tests (input infrastructure, no reconstruction).

Raw word: bits [0,11) column, [11,22) row, [22,27) layer, [27,31) charge.
"""
from __future__ import annotations

import numpy as np

PITCH_MM = 0.055


def word(layer: int, row: int, col: int, q: int = 1) -> int:
    return (int(col) & 0x7FF) | ((int(row) & 0x7FF) << 11) | ((int(layer) & 31) << 22) | ((int(q) & 15) << 27)


def pack(events) -> tuple[np.ndarray, np.ndarray]:
    """events: list of lists of uint32 words (or arrays) -> (pixels, offsets)."""
    arrs = [np.asarray(e, np.uint32).ravel() for e in events]
    offsets = np.zeros(len(arrs) + 1, np.uint64)
    offsets[1:] = np.cumsum([len(a) for a in arrs])
    pixels = np.concatenate(arrs).astype(np.uint32) if arrs else np.zeros(0, np.uint32)
    return pixels, offsets


def pixel_of(x_mm: float, y_mm: float) -> tuple[int, int]:
    """(row, col) of the pixel containing the point (x, y)."""
    c = int(np.floor(x_mm / PITCH_MM + 768.0))
    r = int(np.floor(y_mm / PITCH_MM + 768.0))
    return r, c


def line_event(tracks, layers=range(26), z_of_layer=None, q: int = 5, skip=()) -> list:
    """Words for straight lines given as (x0, y0, tx, ty) at z = 0, one pixel per
    plane (pixels outside the sensor or in the beam hole are left out);
    `skip` lists (track index, layer) pairs to leave out."""
    from .gen import layer_z_mm
    z = layer_z_mm() if z_of_layer is None else z_of_layer
    skip = set(skip)
    words = []
    for l in sorted(layers):
        for i, (x0, y0, tx, ty) in enumerate(tracks):
            if (i, l) in skip:
                continue
            r, c = pixel_of(x0 + tx * z[l], y0 + ty * z[l])
            if not (0 <= r < 1536 and 0 <= c < 1536):
                continue
            if (2 * c - 1535) ** 2 + (2 * r - 1535) ** 2 <= 34393:
                continue
            words.append(word(l, r, c, q))
    return words


def shuffle_within_layers(pixels: np.ndarray, offsets: np.ndarray, seed: int) -> np.ndarray:
    """Random permutation of each event's words that keeps the layer grouping."""
    rng = np.random.default_rng(seed)
    out = pixels.copy()
    for e in range(len(offsets) - 1):
        a, b = int(offsets[e]), int(offsets[e + 1])
        w = out[a:b]
        lay = (w >> 22) & 31
        k = rng.random(len(w))
        out[a:b] = w[np.lexsort((k, lay))]
    return out


def hit_event(planes: dict, n_slots: int | None = None) -> tuple[dict, np.ndarray]:
    """One event of hand-placed hits in the hit layout that clustering writes,
    for feeding track finding directly.

    planes: {plane: [(x_mm, y_mm, id), ...]}; a hit's key is plane << 22 | id
    (ids unique inside a plane).  Hits of a plane are stored by ascending key.
    n_slots (default: the number of hits) sets offsets[1], the event's slot
    range, which also fixes its track capacity floor(n_slots / 3).
    Returns (hits, offsets) with hits = dict(x, y, key, aux, layer_start[1, 27],
    layer_nhits[1, 26], n_hits[1], status[1])."""
    rows = []
    for l in sorted(planes):
        for x, y, i in sorted(planes[l], key=lambda h: h[2]):
            rows.append((l, np.float32(x), np.float32(y), (int(l) << 22) | int(i)))
    n = len(rows)
    N = max(n if n_slots is None else int(n_slots), n, 1)
    x = np.zeros(N, np.float32)
    y = np.zeros(N, np.float32)
    key = np.zeros(N, np.uint32)
    for k, (l, xv, yv, kv) in enumerate(rows):
        x[k], y[k], key[k] = xv, yv, kv
    nh = np.zeros((1, 26), np.uint32)
    for l, *_ in rows:
        nh[0, l] += 1
    ls = np.zeros((1, 27), np.uint32)
    ls[0, 1:] = np.cumsum(nh[0])
    ls[0, 26] = N
    hits = dict(x=x, y=y, key=key, aux=np.full(N, (1 << 16) | 1, np.uint32), layer_start=ls,
                layer_nhits=nh, n_hits=np.array([n], np.uint32), status=np.zeros(1, np.uint32))
    return hits, np.array([0, N], np.uint64)


def bad_offsets_case():
    """Three generated events A, B, C packed back to back, and offset tables,
    each with the status every event must get (32 = bad offsets): a
    decreasing pair, a start below an earlier offset (the words would overlap
    A's), an end beyond the buffer, a repeated offset (an empty event)."""
    from .gen import generate
    b = generate("cpu10", 3)
    nA, nB, nC = (int(b.offsets[e + 1] - b.offsets[e]) for e in range(3))
    N = nA + nB + nC
    cases = {
        # A | B | C, all fine
        "good": ([0, nA, nA + nB, N], [0, 0, 0]),
        # A, then a decreasing pair, then an event inside A's words, then the rest
        "descent": ([0, nA, 40, 50, N], [0, 32, 32, 32]),
        # A twice (the second start lies below the first event's end), C
        "overlap": ([0, nA, 10, nA + nB, N], [0, 32, 32, 0]),
        # A, B, then an end beyond the buffer
        "beyond": ([0, nA, nA + nB, N + 5], [0, 0, 32]),
        # an empty event at a repeated offset is fine
        "empty": ([0, nA, nA, nA + nB, N], [0, 0, 0, 0]),
    }
    return b, cases
