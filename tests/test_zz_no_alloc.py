"""The entry point that allocates nothing (mapper_knn_d2_noalloc) against the
k-NN entry point it mirrors (mapper_knn_d2), through the C ABI (needs an
MI355X).

Both compute the exact k-th nearest-neighbour squared distances (the
eps-selection module of the Use Cases section) with the same kernels; the
no-alloc form keeps its work arrays in the library's static scratch array
instead of the context arena.  Two calls in a row, the second smaller, must
each equal the arena form bit for bit (the array keeps the first call's
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
        for n, d, k in ((20000, 256, 5), (3001, 64, 16)):
            print(f"[case] noalloc knn n={n} d={d} k={k}", flush=True)
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
