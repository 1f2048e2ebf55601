"""The allocation-free batch entry point (rawalign_dtw_batch_noalloc, for
callers that cannot allocate device memory) against the allocating one
(rawalign_dtw_batch_ex with default options) and the oracle, through the C
ABI: two calls in a row on the same fixed scratch, the second smaller."""
import numpy as np
import pytest

from paper_2310_05037_amd import workloads as W

from . import parity

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_2310_05037_amd import lib
    assert torch.cuda.is_available()
    lib.load()
    return lib


def _say(msg):
    print(msg, flush=True)


def _mixed(seed, groups):
    """Pairs over every route: groups of (count, n range, m range); one
    extra pair with an empty query and one with an empty region."""
    rng = np.random.default_rng(seed)
    reads, pairs, r_parts, off = [], [], [], 0
    for count, (n0, n1), (m0, m1) in groups:
        for _ in range(count):
            n = int(rng.integers(n0, n1 + 1))
            m = int(rng.integers(m0, m1 + 1))
            reads.append(rng.standard_normal(n).astype(np.float32))
            r_parts.append(rng.standard_normal(m).astype(np.float32))
            pairs.append((len(reads) - 1, off, m, False))
            off += m
    reads.append(np.zeros(0, np.float32))
    pairs.append((len(reads) - 1, 0, 10, False))        # empty query: (0, -1)
    reads.append(rng.standard_normal(5).astype(np.float32))
    pairs.append((len(reads) - 1, 0, 0, False))         # empty region: (+inf, -1)
    return W._pack(f"noalloc_mixed_{seed}", reads, pairs, np.concatenate(r_parts), {})


def _both(L, b):
    """(noalloc scores, ends), (batch_ex scores, ends) on the same inputs."""
    db = L.DeviceBatch(b)
    _say(f"  gpu: noalloc {b.name} pairs={b.n_pairs} max_n={int(b.q_len.max())} max_m={int(b.r_len.max())}")
    L.rawalign_dtw_batch_noalloc(*db.args())
    got = db.results()
    got = (got[0].copy(), got[1].copy())
    _say(f"  gpu: batch_ex {b.name}")
    db.run(opts=L.make_opts())
    ref = db.results()
    return got, ref


def test_noalloc_equals_batch_ex_two_calls(L):
    """First call: every route, with more regions above 4096 levels than the
    fixed edge slots (waves reuse their slot through the queue).  Second
    call: a smaller batch on the same scratch, which keeps the first call's
    contents.  Both equal rawalign_dtw_batch_ex bit for bit and the float
    oracle bit for bit (within 1e-4 of the double oracle)."""
    first = _mixed(1, [(300, (1, 400), (1, 2048)), (100, (1, 300), (2049, 4096)),
                       (L.RAWALIGN_NOALLOC_EDGE_SLOTS + 188, (1, 120), (4097, 12000))])
    second = _mixed(2, [(150, (1, 200), (1, 6000)), (20, (60, 300), (4097, 20000))])
    assert second.n_pairs < first.n_pairs
    for b in (first, second):
        (s, e), (rs, re_) = _both(L, b)
        assert np.array_equal(s.view(np.uint32), rs.view(np.uint32)) and np.array_equal(e, re_), b.name
        st = parity.check(b, s, e)
        print(b.name, st)
        assert s[-2] == 0.0 and e[-2] == -1 and np.isinf(s[-1]) and e[-1] == -1


def test_noalloc_rejects_too_many_pairs(L):
    """n_pairs beyond the fixed scratch is refused before anything runs."""
    import torch
    n = L.RAWALIGN_NOALLOC_MAX_PAIRS + 1
    dev = "cuda"
    q = torch.zeros(4, dtype=torch.float32, device=dev)
    off = torch.zeros(n, dtype=torch.int64, device=dev)
    ln = torch.ones(n, dtype=torch.int32, device=dev)
    out = torch.empty(n, dtype=torch.float32, device=dev)
    end = torch.empty(n, dtype=torch.int32, device=dev)
    with pytest.raises(L.RawAlignError) as ei:
        L.rawalign_dtw_batch_noalloc(q, off, ln, q, off, ln, out, end)
    assert ei.value.code == L.RAWALIGN_EINVAL and "exceeds" in str(ei.value)
