"""velo_reconstruct_noalloc, the allocation-free form of velo_reconstruct
(its workspace is the library's own device array): through the C ABI, two
calls in a row, the second on a smaller batch, each equal to
velo_reconstruct with a caller workspace on the same input (hits, tracks
and their order bit for bit, states within the parity tolerance) and to the
oracle."""
import numpy as np
import pytest

from gpu_helpers import compare_all, host, to_dev
from synth import generate

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_noalloc_equals_reconstruct(orc):
    import torch

    import paper_1912_09161_amd as velo
    batches = [generate("nominal", 400, first_event=2000, workers=8),
               generate("uneven", 150, first_event=3000, workers=8)]
    assert batches[1].n_pixels < batches[0].n_pixels
    stream = torch.cuda.Stream()
    for i, b in enumerate(batches):
        print(f"noalloc call {i}: {b.n_events} events, {b.n_pixels} words", flush=True)
        px, off = to_dev(b.pixels, b.offsets)
        assert velo.workspace_bytes(b.n_pixels, b.n_events) <= velo.NOALLOC_SCRATCH_BYTES
        with torch.cuda.stream(stream):
            ref = velo.reconstruct(px, off, stream=stream)
            got = velo.reconstruct_noalloc(px, off, stream=stream)
        stream.synchronize()
        g, r = host(got), host(ref)
        compare_all(g, r, b.offsets)
        for part in ("hits", "tracks"):
            for k in ("status", "n_hits", "layer_start", "layer_nhits", "n_tracks"):
                if k in r[part]:
                    np.testing.assert_array_equal(g[part][k], r[part][k], err_msg=k)
        o = orc.reconstruct(b.pixels, b.offsets, threads=8)
        compare_all(g, o, b.offsets)
