"""The allocation-free codec entry point (codec_encode_noalloc, workspace in
the library's static device scratch) gives the same stream as codec_encode
with a caller workspace, on two calls in a row (the second with a smaller
input, over the scratch the first left behind), and rejects inputs larger
than its scratch holds."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_14088_amd import bmq  # noqa: E402

DEV = "cuda:0"


def planes(n, seed):
    rng = np.random.default_rng(seed)
    scale = 2.0 ** rng.uniform(-30, 0, n)
    re = (rng.standard_normal(n) * scale).astype(np.float32)
    im = (rng.standard_normal(n) * scale).astype(np.float32)
    re[64:192] = 0.0
    return torch.from_numpy(re).to(DEV), torch.from_numpy(im).to(DEV)


@pytest.mark.parametrize("domain", [0, 1])
def test_noalloc_encode_matches_workspace_encode(domain):
    cfg = bmq.Config(n=10, b=10, domain=domain, eb=1e-5)
    for n, seed in ((1 << 24, 1), (64 * 777, 2)):          # full scratch, then a smaller input
        print(f"noalloc n={n} domain={domain}", flush=True)
        re, im = planes(n, seed + 10 * domain)
        want = bmq.codec_encode(re, im, cfg)
        got = bmq.codec_encode_noalloc(re, im, cfg)
        torch.cuda.synchronize()
        assert got.numel() == want.numel()
        assert torch.equal(got, want)
        r2, i2 = bmq.codec_decode(got, n, cfg)
        r3, i3 = bmq.codec_decode(want, n, cfg)
        assert torch.equal(r2.view(torch.int32), r3.view(torch.int32))
        assert torch.equal(i2.view(torch.int32), i3.view(torch.int32))


def test_noalloc_rejects_inputs_beyond_its_scratch():
    cfg = bmq.Config(n=10, b=10, domain=1, eb=1e-5)
    n = (1 << 24) + 64
    x = torch.zeros(n, dtype=torch.float32, device=DEV)
    with pytest.raises(bmq.BmqError) as e:
        bmq.codec_encode_noalloc(x, x, cfg, cap=64)
    assert e.value.code == -1 and "static scratch" in str(e.value)
