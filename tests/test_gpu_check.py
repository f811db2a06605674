"""Directory validation (sv_check) on the GPU.

Valid states of every kind pass with no bad entry: LIN, LOG and RAW
domains, records in the device pool and in the pinned host pool, the initial
state.  A directory entry corrupted from the host (through the read-only view
sv_directory gives, written via the arena that holds it) is caught:
an impossible width, a sign class in a LIN state, a packed plane in a RAW
state, a record beyond its pool, the overflow marker.  The state is then
poisoned (SV_ERR_CORRUPT, later calls refuse), and a reset state passes
again.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2410_14088_amd import bmq  # noqa: E402
from paper_2410_14088_amd import circuits as C  # noqa: E402

DEV = "cuda:0"
OFF_MASK = (1 << 40) - 1


def _state(domain=1, **kw):
    d = C.config(0)
    cfg = bmq.Config(n=d["n"], b=d["b"], inner=2, fuse=2, domain=domain, eb=1e-5 if domain != 0 else 1e-6, **kw)
    plan = bmq.Plan(d["gates"][:120], cfg)
    sv = bmq.State(cfg, DEV)
    return sv, plan


def _dir_view(sv):
    ptr, n = sv.directory()
    off = ptr - sv.arena.data_ptr()
    assert off >= 0 and off % 8 == 0 and off + 8 * n <= sv.arena.numel()
    return sv.arena[off:off + 8 * n].view(torch.int64)


def _u64(x):
    return int(x) & ((1 << 64) - 1)


def _i64(x):
    x &= (1 << 64) - 1
    return x - (1 << 64) if x >= 1 << 63 else x


@pytest.mark.parametrize("domain", [0, 1, 2])
def test_valid_states_pass(domain):
    sv, plan = _state(domain)
    print(f"domain {domain}: initial state and after 120 gates", flush=True)
    assert sv.check() == 0
    sv.apply(plan)
    assert sv.check() == 0
    d = _dir_view(sv).cpu().numpy().view(np.uint64)
    assert np.count_nonzero(d) > 0


def test_host_pool_records_pass():
    sv0, plan = _state(1)
    st = sv0.apply(plan, stats=True)
    peak = max(x["bytes_out"] for x in st)
    sv, plan = _state(1, pool_bytes=peak // 4)
    sv.attach_host_pool(4 * peak)
    print("records in the host pool", flush=True)
    sv.apply(plan)
    assert sv.footprint()[1] > 0
    assert sv.check() == 0


def _corrupt_and_check(sv, mutate, label):
    dv = _dir_view(sv)
    d = dv.cpu().numpy().view(np.uint64)
    k = int(np.flatnonzero(d)[len(np.flatnonzero(d)) // 2])
    e = _u64(d[k])
    dv[k] = _i64(mutate(e))
    torch.cuda.synchronize()
    print(f"corruption: {label} at chunk {k}", flush=True)
    with pytest.raises(bmq.BmqError) as ei:
        sv.check()
    assert ei.value.code == -5
    with pytest.raises(bmq.BmqError):              # poisoned
        sv.fidelity(None)
    sv.reset()                                     # a fresh |0...0> is valid again
    assert sv.check() == 0


def _with_header(e, h0):
    return (e & ~(0xFFF << 40)) | (h0 << 40)


@pytest.mark.parametrize("case", ["width", "beyond_pool", "overflow_marker", "zero_headers"])
def test_corrupt_entries_are_caught(case):
    sv, plan = _state(1)
    sv.apply(plan)
    assert sv.check() == 0
    if case == "width":
        mutate = lambda e: _with_header(e, 1 | (40 << 2))               # LZ plane of width 40
    elif case == "beyond_pool":
        mutate = lambda e: (e & ~OFF_MASK) | (OFF_MASK - 8)              # no pool reaches there
    elif case == "overflow_marker":
        mutate = lambda e: (1 << 64) - 1
    else:
        mutate = lambda e: (e & OFF_MASK) | 64                           # offset without headers
    _corrupt_and_check(sv, mutate, case)


def test_domain_specific_headers_are_caught():
    # a sign class is impossible in LIN, a packed plane in RAW
    sv, plan = _state(0)
    sv.apply(plan)
    _corrupt_and_check(sv, lambda e: _with_header(e, 1 | (3 << 2) | (2 << 8)), "LIN sign class")
    sv, plan = _state(2)
    sv.apply(plan)
    _corrupt_and_check(sv, lambda e: _with_header(e, 2 | (5 << 2)), "RAW packed plane")
