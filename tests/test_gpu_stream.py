"""The bandwidth probes (ipm_stream_read, ipm_stream_copy): the read pass returns the FP64 sum of
its buffer (checked against an exactly rounded host sum within the bound of any summation order),
the copy pass reproduces its source bit for bit, including ragged lengths that leave a partial
pass, a partial 16-byte word or an odd FP64 word; bad arguments are rejected before any launch."""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P = None


@pytest.fixture(scope="module")
def ctx():
    global P
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2209_08722_amd as mod
    P = mod
    c = mod.Context(0)
    yield c
    torch.cuda.synchronize()
    c.close()


@pytest.mark.parametrize("count", [0, 1, 2, 3, 1023, 2048, 2049, 4097, 1_000_003, 8_388_608 + 5])
def test_stream_read_sum(ctx, count):
    rng = np.random.default_rng(count)
    x = rng.standard_normal(count)
    got = float(P.ipm_stream_read(ctx, torch.from_numpy(x).to("cuda:0")).cpu()[0])
    exact = math.fsum(x.tolist()) if count else 0.0
    # any order of count - 1 FP64 additions is within (count - 1) u sum |x| of the exact sum
    assert abs(got - exact) <= max(count - 1, 0) * 2.0 ** -53 * float(np.abs(x).sum()) * 1.01


def test_stream_read_reproducible(ctx):
    x = torch.randn(3_000_001, dtype=torch.float64, device="cuda:0")
    a = P.ipm_stream_read(ctx, x).cpu()
    b = P.ipm_stream_read(ctx, x).cpu()
    assert a.item() == b.item()


@pytest.mark.parametrize("nbytes", [0, 1, 15, 16, 17, 32768, 32768 + 16 * 7 + 9, 10_000_007, 64 << 20])
def test_stream_copy_exact(ctx, nbytes):
    g = torch.Generator(device="cuda:0")
    g.manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes + 64,), dtype=torch.uint8, device="cuda:0", generator=g)
    dst = torch.zeros(nbytes + 64, dtype=torch.uint8, device="cuda:0")
    P.ipm_stream_copy(ctx, src, dst, nbytes)
    torch.cuda.synchronize()
    assert torch.equal(dst[:nbytes], src[:nbytes])
    assert int(dst[nbytes:].count_nonzero()) == 0          # nothing written past the end


def test_stream_probe_arguments(ctx):
    x = torch.zeros(1024, dtype=torch.float64, device="cuda:0")
    with pytest.raises(P.IpmError):
        P.ipm_stream_read(ctx, x[1:])                        # 8-byte offset: not 16-byte aligned
    b = torch.zeros(4096, dtype=torch.uint8, device="cuda:0")
    with pytest.raises(P.IpmError):
        P.ipm_stream_copy(ctx, b[:2048], b[16:], 2048)       # overlapping ranges
    with pytest.raises(P.IpmError):
        P.ipm_stream_copy(ctx, b[8:1032], b[2048:3072], 1024)   # misaligned source
    rc = ctx.lib.ipm_stream_read(ctx.h, x.data_ptr(), -1, x.data_ptr())
    assert rc == P.native.IPM_ERR_ARG
    torch.cuda.synchronize()
