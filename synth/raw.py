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
