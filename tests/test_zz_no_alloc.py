"""The entry point that allocates nothing (mapper_knn_d2_noalloc) against the
k-NN entry point it mirrors (mapper_knn_d2), through the C ABI (needs an
MI355X).

Both compute the exact k-th nearest-neighbour squared distances (the
eps-selection module of the Use Cases section) with the same kernels; the
no-alloc form keeps its work arrays in the library's static scratch array
instead of the context arena.  Calls in a row, each smaller than the one
before, must each equal the arena form bit for bit (the array keeps the first call's
contents); an input too large for the array is refused before any launch.
"""
import numpy as np
import pytest

from paper_2011_03209_amd import binding, synth

pytestmark = pytest.mark.gpu


def test_noalloc_knn_matches_arena_form():
    import torch
    ctx = binding.Context(arena_bytes=1 << 30)
    try:
        rng = np.random.default_rng(4242)
        # the third: 1100 exact copies of two points, more candidates per row
        # than the first lists hold, so pass 2 runs again in both forms
        for n, d, k, copies in ((20000, 256, 5, 1), (3001, 64, 16, 1), (2200, 16, 5, 1100)):
            print(f"[case] noalloc knn n={n} d={d} k={k} copies={copies}", flush=True)
            if copies > 1:
                X = np.repeat(rng.normal(size=(n // copies, d)).astype(np.float32), copies, axis=0)
            else:
                X, _ = synth.gaussian_mixture(rng, n, d, 12)
            cloud = ctx.cloud(X)
            try:
                ref, _ = cloud.knn_d2(k)
            finally:
                cloud.destroy()
            pts = torch.from_numpy(X).to("cuda")
            out = torch.full((n,), -1.0, dtype=torch.float64, device="cuda")
            used0 = ctx.memory()[0]
            ctx.knn_d2_noalloc(pts, k, out)
            torch.cuda.synchronize()
            assert ctx.memory()[0] == used0                 # nothing taken from the arena
            got = out.cpu().numpy()
            assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
        # past the array's capacity: refused with a message, nothing launched
        big = torch.zeros((400000, 256), dtype=torch.float32, device="cuda")
        out = torch.zeros(400000, dtype=torch.float64, device="cuda")
        with pytest.raises(binding.MapperError, match="no-alloc scratch"):
            ctx.knn_d2_noalloc(big, 5, out)
    finally:
        ctx.close()
