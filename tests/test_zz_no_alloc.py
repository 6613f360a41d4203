"""The allocation-free entry point care_gram_noalloc against care_gram,
through the C ABI: two calls in a row on one context (the second smaller, so
stale partial sums of the first call in the fixed device array would show),
elementwise within the FP64 rounding bound of the two summation orders;
size limits rejected before any device work."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def pk():
    import paper_2607_14742_amd as pk
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pk.load()
    return pk


def _cm(rows, cols, gen):
    # column-major n x k FP64 on the GPU
    return torch.randn(cols, rows, dtype=torch.float64, generator=gen).t().cuda()


@pytest.mark.parametrize("allocator", ["torch", None])
def test_gram_noalloc_matches_gram(pk, allocator):
    gen = torch.Generator().manual_seed(1220)
    ctx = pk.Context(0, allocator=allocator)
    try:
        # (n, a, b): ragged row count and tile edges; the second call smaller
        for n, a, b in ((250_003, 403, 397), (1_000, 37, 5)):
            print(f"gram_noalloc n={n} a={a} b={b}", flush=True)
            X = _cm(n, a, gen)
            Y = _cm(n, b, gen)
            C0 = pk.gram(ctx, X, Y)
            C1 = pk.gram_noalloc(ctx, X, Y)
            bound = 2.0 * n * np.finfo(np.float64).eps * (X.abs().t() @ Y.abs())
            err = (C1 - C0).abs()
            assert bool((err <= bound).all()), float((err / bound).max())
            # the Gram of a matrix with itself (every tile computed, no mirror)
            G0 = pk.gram(ctx, X, X)
            G1 = pk.gram_noalloc(ctx, X, X)
            bound = 2.0 * n * np.finfo(np.float64).eps * (X.abs().t() @ X.abs())
            assert bool(((G1 - G0).abs() <= bound).all())
    finally:
        ctx.close()


def test_gram_noalloc_rejects_sizes_beyond_the_array(pk):
    ctx = pk.Context(0)
    try:
        X = torch.zeros(10, 2049, dtype=torch.float64, device="cuda")     # ceil(2049/32)^2 = 4225 > 4096 tiles
        with pytest.raises(pk.CareError) as e:
            pk.gram_noalloc(ctx, X, X)
        assert e.value.name == "CARE_ERR_ARG"
    finally:
        ctx.close()
