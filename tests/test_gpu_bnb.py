"""GPU parity of mapping with early termination (rawalign_map_bnb): the
per-read decision equals the oracle's decision over every candidate's full
DTW; completed candidates equal the float oracle bit for bit; every dropped
candidate's full Score is below its read's best (so dropping it was safe)."""
import numpy as np
import pytest

from oracle import oracle
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


def _run_bnb(L, b, max_query=None, block_rows=512, b_match=0.4, threshold=20.0, cand_cnt=None):
    import torch
    dev = "cuda"
    db = L.DeviceBatch(b)
    n_reads = len(b.cand_off)
    row_off = np.concatenate([[0], np.cumsum(b.r_len.astype(np.int64))[:-1]]).astype(np.int64)
    rows = torch.empty(int(b.r_len.astype(np.int64).sum()) + 1, dtype=torch.float32, device=dev)
    cc = b.cand_cnt if cand_cnt is None else cand_cnt
    ob = torch.empty(n_reads, dtype=torch.int32, device=dev)
    os_ = torch.empty(n_reads, dtype=torch.float64, device=dev)
    om = torch.empty(n_reads, dtype=torch.uint8, device=dev)
    mq = int(b.q_len.max()) if max_query is None else max_query
    _say(f"  gpu: bnb {b.name} pairs={b.n_pairs} reads={n_reads} max_query={mq} block_rows={block_rows}")
    L.rawalign_map_bnb(db.q, db.q_off, db.q_len, db.r, db.r_off, db.r_len,
                       torch.from_numpy(b.cand_off).to(dev), torch.from_numpy(np.ascontiguousarray(cc)).to(dev),
                       torch.from_numpy(b.n_events).to(dev), rows, torch.from_numpy(row_off).to(dev),
                       db.score, db.end, ob, os_, om, max_query=mq, block_rows=block_rows, b_match=b_match,
                       threshold=threshold)
    s, e = db.results()
    return s, e, ob.cpu().numpy(), os_.cpu().numpy(), om.cpu().numpy()


def _check(b, s, e, ob, os_, om, s32, e32, b_match=0.4, threshold=20.0, cand_cnt=None):
    cc = b.cand_cnt if cand_cnt is None else cand_cnt
    rb, rs, rm = oracle.decide(s32, b.cand_off, cc, b.n_events, b_match, threshold)
    assert np.array_equal(ob, rb)
    assert np.array_equal(os_.view(np.uint64), rs.view(np.uint64))
    assert np.array_equal(om, rm)
    pruned = e == -3
    done = ~pruned
    assert np.array_equal(s[done].view(np.uint32), s32[done].view(np.uint32))
    assert np.array_equal(e[done], e32[done])
    assert np.isinf(s[pruned]).all()
    # a dropped pair's full Score is strictly below its read's best
    for k in range(len(b.cand_off)):
        p0, cnt = int(b.cand_off[k]), int(cc[k])
        for p in range(p0, p0 + cnt):
            if pruned[p]:
                assert b_match * float(b.n_events[k]) - float(s32[p]) < rs[k], (k, p)
    return int(pruned.sum())


def test_bnb_uneven_batch_matches_full_decision(L):
    """2,000 pairs of the uneven workload (1-50 candidates per read, regions
    up to 3x the read, multi-stripe regions, queries over several blocks),
    candidates in a synthetic chaining order."""
    b = W.chain_ordered(W.uneven_batch(n_pairs=2000), seed=1)
    s32, e32, _ = oracle.dtw_batch_f32(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, parity.threads())
    for block_rows in (512, 64):
        s, e, ob, os_, om = _run_bnb(L, b, block_rows=block_rows)
        n_pruned = _check(b, s, e, ob, os_, om, s32, e32)
        print("bnb", block_rows, "pruned", n_pruned, "of", b.n_pairs)
        assert n_pruned > 0


def test_bnb_edge_cases(L):
    """A read without candidates, reads sharing a pair, a query longer than
    max_query, degenerate pairs, another match bonus and threshold."""
    b = W.chain_ordered(W.plain_batch(n_pairs=400), seed=2)
    q_len = b.q_len.copy()
    b = W.Batch(b.name, b.q, b.r, b.q_off, q_len, b.r_off, b.r_len.copy(), b.cand_off, b.cand_cnt,
                b.n_events, b.true_pair, b.meta)
    b.r_len[7] = 0                                  # empty region
    b.q_len[11] = 0                                 # empty query
    cc = b.cand_cnt.copy()
    cc[3] = 0                                       # a read without candidates
    cc[5] = cc[5] + 2 if b.cand_off[5] + cc[5] + 2 <= b.n_pairs else cc[5]   # overlaps read 6
    max_query = int(b.q_len.max()) - 1             # the longest read's queries exceed it
    over = b.q_len > max_query                      # all candidates of that read share its query
    s32, e32, _ = oracle.dtw_batch_f32(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, parity.threads())
    s32 = s32.copy()
    e32 = e32.copy()
    s32[over] = np.nan
    e32[over] = -2
    for bm, th in ((0.4, 20.0), (0.3, 5.0)):
        s, e, ob, os_, om = _run_bnb(L, b, max_query=max_query, block_rows=128, b_match=bm, threshold=th,
                                     cand_cnt=cc)
        assert np.isnan(s[over]).all() and (e[over] == -2).all()
        assert s[7] == np.inf and e[7] == -1 and s[11] == 0.0 and e[11] == -1
        keep = ~over
        # reads holding an over-long query decide on NaN; compare the others
        rb, rs, rm = oracle.decide(s32, b.cand_off, cc, b.n_events, bm, th)
        ok_reads = np.array([not over[int(b.cand_off[k]):int(b.cand_off[k] + cc[k])].any() for k in range(len(cc))])
        assert np.array_equal(ob[ok_reads], rb[ok_reads])
        assert np.array_equal(os_[ok_reads].view(np.uint64), rs[ok_reads].view(np.uint64))
        assert np.array_equal(om[ok_reads], rm[ok_reads])
        done = (e != -3) & keep
        assert np.array_equal(s[done].view(np.uint32), s32[done].view(np.uint32))
        # pairs of reads 5 and 6 that both claim are never dropped
        shared = range(int(b.cand_off[6]), int(b.cand_off[5] + cc[5]))
        assert all(e[p] != -3 for p in shared)


def _long_candidates(seed=7, n_reads=12, cands=5):
    """Reads of 2,500-6,000 events, each with 5 candidate regions of
    8,000-20,000 levels (4 to 10 stripes, over 2e7 cells per pair): the
    true region at position k % cands of read k (first, middle, last),
    read 0 all decoys."""
    rng = np.random.default_rng(seed)
    model = W.pore_model(rng)
    bases = W.random_bases(rng, 2_000_000)
    r = W.expected_levels(bases, model)
    L = len(r)
    reads, pairs = [], []
    for k in range(n_reads):
        n = int(rng.integers(2500, 6001))
        start = int(rng.integers(0, L - 4 * n))
        ev, span = W.read_events(rng, r, start, n_events=n)
        reads.append(ev)
        true_at = k % cands
        for c in range(cands):
            m = int(rng.integers(8000, 20001))
            if c == true_at and k != 0:
                pairs.append((k, W._true_region(rng, start, span, m, L), m, True))
            else:
                pairs.append((k, int(rng.integers(0, L - m + 1)), m, False))
    return W._pack("long_candidates", reads, pairs, r, {})


def test_bnb_long_candidates(L):
    """Long candidates only (several stripes and many row blocks per pair,
    true regions before, among and after decoys): decisions equal the
    oracle's over full scores, completed pairs equal the float oracle bit
    for bit, drops are justified, for two block sizes (one not dividing the
    queries)."""
    b = _long_candidates()
    assert (b.r_len > 4096).all() and (b.q_len.astype(np.int64) * b.r_len >= 20_000_000).all()
    s32, e32, _ = oracle.dtw_batch_f32(b.q, b.q_off, b.q_len, b.r, b.r_off, b.r_len, parity.threads())
    for block_rows in (512, 200):
        s, e, ob, os_, om = _run_bnb(L, b, block_rows=block_rows)
        n_pruned = _check(b, s, e, ob, os_, om, s32, e32)
        print("long", block_rows, "pruned", n_pruned, "of", b.n_pairs, "mapped", int(om.sum()))
        assert n_pruned > 0 and not np.isnan(s).any()
