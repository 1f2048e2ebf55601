"""Graph capture of the banded and warping-path entry points: each is
captured once into a HIP graph (after a warm-up call on the same stream,
which allocates the library's scratch), then replayed three times with
other device work and host synchronisations in between; every replay must
reproduce the eager results bit for bit."""
import numpy as np
import pytest

from paper_2310_05037_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def L():
    import torch
    from paper_2310_05037_amd import lib
    assert torch.cuda.is_available()
    lib.load()
    return lib


def _replays(fn, outs):
    """Capture fn on a side stream, then check three replays against the
    eager results (outs: the tensors fn writes)."""
    import torch
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        fn(st)
        st.synchronize()
        ref = [o.clone() for o in outs]
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=st):
            fn(st)
    for k in range(3):
        for o in outs:
            o.fill_(-9)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o.view(torch.int32), r.view(torch.int32)), k


def test_band_graph_replay(L):
    import torch
    rng = np.random.default_rng(41)
    b = W.random_pairs(rng, 400, (20, 900), (1, 1200))
    band = torch.from_numpy(rng.integers(0, 300, size=b.n_pairs).astype(np.int32)).cuda()
    db = L.DeviceBatch(b)
    print(f"  gpu: band graph pairs={b.n_pairs}", flush=True)
    _replays(lambda st: L.rawalign_dtw_band(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, band, db.score,
                                            db.end, stream=st), [db.score, db.end])


def test_path_graph_replay(L):
    import torch
    rng = np.random.default_rng(42)
    b = W.random_pairs(rng, 200, (1, 700), (1, 3000))
    db = L.DeviceBatch(b)
    dir_off, words = L.path_workspace(b.q_len, b.r_len)
    dir_off = torch.from_numpy(dir_off).cuda()
    dirs = torch.empty(words, dtype=torch.int64, device="cuda")
    rows = b.q_len.astype(np.int64)
    path_off = torch.from_numpy(np.concatenate([[0], np.cumsum(rows)[:-1]]).astype(np.int64)).cuda()
    lo = torch.empty(int(rows.sum()), dtype=torch.int32, device="cuda")
    hi = torch.empty_like(lo)
    start = torch.empty(b.n_pairs, dtype=torch.int32, device="cuda")
    print(f"  gpu: path graph pairs={b.n_pairs}", flush=True)
    _replays(lambda st: L.rawalign_dtw_path(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len, dir_off, dirs,
                                            path_off, lo, hi, db.score, db.end, start, stream=st),
             [db.score, db.end, start, lo, hi])
