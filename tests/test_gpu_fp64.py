"""The FP64 square root on the GPU at scale (needs an MI355X).

Bit-exact binning under the L2 lens and under the whole-cloud lenses (k-NN
distance, eccentricity) depends on the GPU's FP64 square root being correctly
rounded, as IEEE 754 requires of the host's (Background section: the filter
function; the L2 norm is one of the paper's filters).  These tests compare
the library's square root kernel with numpy's (the host's correctly rounded
sqrt) on 1e8 inputs -- random doubles over the whole exponent range, exact
squares, values whose root lies within a quarter ulp of a rounding midpoint,
subnormals and other edge values -- and the L2 lens of a 2e7-point cloud with
the oracle's, bit for bit.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_03209_amd import synth

pytestmark = pytest.mark.gpu

CHUNK = 25_000_000


@pytest.fixture(scope="module")
def ctx():
    from paper_2011_03209_amd import binding
    c = binding.Context(arena_bytes=4 << 30)
    yield c
    c.close()


def _random_doubles(rng, n):
    """Positive doubles, uniform 52-bit fractions, exponents over the normal range."""
    frac = rng.integers(0, 1 << 52, size=n, dtype=np.uint64)
    expo = rng.integers(1, 2047, size=n, dtype=np.uint64)
    return ((expo << np.uint64(52)) | frac).view(np.float64)


def _exact_squares(rng, n):
    """y * y with y of at most 26 significant bits: the product is exact and
    its square root is y itself."""
    m = rng.integers(1 << 25, 1 << 26, size=n, dtype=np.int64).astype(np.float64)
    e = rng.integers(-480, 480, size=n)
    y = np.ldexp(m, e - 25)
    return y * y


def _near_midpoints(rng, n):
    """For random y, the double nearest to (y + ulp(y)/2)^2 and its two
    neighbours: their square roots lie within about a quarter ulp of the
    midpoint between y and the next double, so rounding them right needs
    more than the 53 + 2 bits a careless refinement keeps."""
    k = n // 3
    y = _random_doubles(rng, k)
    y = np.ldexp(1.0 + (y.view(np.uint64) & np.uint64((1 << 52) - 1)).astype(np.float64) * 2.0 ** -52,
                 rng.integers(-500, 500, size=k))
    up = np.nextafter(y, np.inf)
    mid_lo = y.astype(np.longdouble) + (up.astype(np.longdouble) - y.astype(np.longdouble)) / 2
    s = (mid_lo * mid_lo).astype(np.float64)
    out = np.concatenate([s, np.nextafter(s, 0.0), np.nextafter(s, np.inf)])
    return out[:n] if out.size >= n else np.concatenate([out, _random_doubles(rng, n - out.size)])


def _edge_values(rng, n):
    tiny = np.float64(np.finfo(np.float64).tiny)
    special = [0.0, tiny, np.nextafter(tiny, 0.0), np.nextafter(0.0, 1.0), np.finfo(np.float64).max,
               1.0, np.nextafter(1.0, 2.0), np.nextafter(1.0, 0.0), 2.0, 4.0, 0.25, 3.0]
    pw = np.ldexp(1.0, np.arange(-1074, 1024))
    sub = (rng.integers(1, 1 << 52, size=n // 4, dtype=np.uint64)).view(np.float64)   # subnormals
    near1 = 1.0 + (rng.integers(-4096, 4096, size=n // 4)).astype(np.float64) * 2.0 ** -52
    ints = rng.integers(0, 1 << 53, size=n // 4).astype(np.float64)                     # integer sums of squares
    out = np.concatenate([np.array(special), pw, sub, near1, ints])
    return np.concatenate([out, _random_doubles(rng, n - out.size)]) if out.size < n else out[:n]


@pytest.mark.parametrize("kind", ["random", "exact_squares", "near_midpoints", "edges"])
def test_sqrt_correctly_rounded(ctx, kind):
    """1e8 inputs in total (2.5e7 per kind), every result bit-identical to the
    host's correctly rounded square root."""
    rng = np.random.default_rng({"random": 1, "exact_squares": 2, "near_midpoints": 3, "edges": 4}[kind])
    gen = {"random": _random_doubles, "exact_squares": _exact_squares, "near_midpoints": _near_midpoints,
           "edges": _edge_values}[kind]
    x = gen(rng, CHUNK)
    assert x.size == CHUNK and np.all(x >= 0) and np.all(np.isfinite(x))
    print(f"[case] sqrt {kind} n={x.size}", flush=True)
    got = ctx.debug_sqrt(x)
    ref = np.sqrt(x)
    bad = np.nonzero(got.view(np.uint64) != ref.view(np.uint64))[0]
    assert bad.size == 0, f"{bad.size} wrong, first x={x[bad[0]]!r} got={got[bad[0]]!r} want={ref[bad[0]]!r}"
    if kind == "exact_squares":
        assert np.array_equal(got * got, x)


def test_l2_lens_at_scale(ctx):
    """The L2 lens of 2e7 points in R^2 through the GPU lens kernel against
    the oracle: random rows of mixed magnitude plus rows (3a, 4a) whose norm
    5|a| is exact, bit for bit."""
    rng = np.random.default_rng(11)
    n = 20_000_000
    X = (rng.standard_normal((n, 2), dtype=np.float32)
         * np.exp2(rng.integers(-30, 30, size=(n, 1))).astype(np.float32))
    a = np.exp2(rng.integers(-20, 20, size=n // 10)).astype(np.float32) * rng.integers(1, 1000, size=n // 10).astype(np.float32)
    X[: n // 10, 0] = 3 * a
    X[: n // 10, 1] = 4 * a
    X = np.ascontiguousarray(X)
    axis = synth.Axis(synth.LENS_L2, 1, 0.0)
    print(f"[case] l2 lens n={n}", flush=True)
    cloud = ctx.cloud(X)
    try:
        got = cloud.debug_lens(axis)
    finally:
        cloud.destroy()
    ref = O.lens(X, axis)
    assert np.array_equal(got.view(np.uint64), ref.view(np.uint64))
    assert np.array_equal(got[: n // 10], 5.0 * a.astype(np.float64))
