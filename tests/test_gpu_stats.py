"""Stage statistics against the directory they describe, on the GPU.

The pass kernel derives most of its statistics instead of counting them per
wave (device bytes from the segment cursors less the spilled bytes, LZ
planes as all planes less the other modes).  After every stage the numbers
sv.apply reports must equal what the live chunk directory says: the mode of
each plane from its header, the all-zero chunks (entry 0), the record bytes
from the headers (body sizes per the record format) and, with a small device
pool and a pinned host pool, the bytes whose offsets address the host pool.
"""
import numpy as np
import pytest

from oracle.mlp import _body_bytes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_14088_amd import bmq  # noqa: E402
from paper_2410_14088_amd import circuits as C  # noqa: E402

DEV = "cuda:0"
OFF_MASK = (1 << 40) - 1


def _entries(sv):
    ptr, n = sv.directory()
    off = ptr - sv.arena.data_ptr()
    assert off >= 0 and off % 8 == 0 and off + 8 * n <= sv.arena.numel()
    return [int(x) & ((1 << 64) - 1) for x in sv.arena[off:off + 8 * n].view(torch.int64).cpu().numpy()]


@pytest.mark.parametrize("domain,spill", [(0, False), (1, False), (1, True)])
def test_stage_statistics_match_the_directory(domain, spill):
    d = C.config(0)                                   # 16 qubits, 2^10-amplitude blocks
    n, b = d["n"], d["b"]
    eb = d["eb"] if domain == 0 else 1e-5
    pool = 0
    if spill:                                         # a quarter of the peak on the device
        cfg0 = bmq.Config(n=n, b=b, inner=2, fuse=2, domain=domain, eb=eb)
        s0 = bmq.State(cfg0, DEV)
        pool = (max(s["bytes_out"] for s in s0.apply(bmq.Plan(d["gates"], cfg0), stats=True)) // 4) & ~255
        s0.close()
    cfg = bmq.Config(n=n, b=b, inner=2, fuse=2, domain=domain, eb=eb, pool_bytes=pool)
    plan = bmq.Plan(d["gates"], cfg)
    sv = bmq.State(cfg, DEV)
    if spill:
        sv.attach_host_pool(16 * pool)
    print(f"domain {domain}, spill {spill}: {plan.n_stages} stages", flush=True)
    host_seen = 0
    for s in range(plan.n_stages):
        st = sv.apply(plan, first=s, count=1, stats=True)[0]
        hist, zero, total, host = [0, 0, 0, 0], 0, 0, 0
        for e in _entries(sv):
            h0, h1 = (e >> 40) & 0xFFF, e >> 52
            hist[h0 & 3] += 1
            hist[h1 & 3] += 1
            zero += e == 0
            size = _body_bytes(h0, h1) + _body_bytes(h1, h0)
            total += size
            if spill and e and (e & OFF_MASK) >= pool:      # offsets at and above the device pool's size
                host += size
        assert st["mode_hist"] == hist, (s, st["mode_hist"], hist)
        assert st["zero_chunks_out"] == zero, s
        assert st["bytes_out"] == total, (s, st["bytes_out"], total)
        assert st["bytes_out_host"] == host, (s, st["bytes_out_host"], host)
        host_seen = max(host_seen, host)
    assert (host_seen > 0) == spill
