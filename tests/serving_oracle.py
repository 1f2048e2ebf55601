"""CPU backend for the serving engine built on the oracle (tests only).

It stores the resident rows in host memory and computes each job with the
float oracle continued from the stored row, so its results are bit-identical
to the GPU's; the decision uses the oracle's Sec. 2.3 rule."""
import numpy as np

from oracle import oracle


class OracleBackend:
    def __init__(self, r_levels, arena_floats, fail_on_call=None):
        self.r = np.ascontiguousarray(r_levels, np.float32)
        self.rows = np.zeros(int(arena_floats), np.float32)
        self.calls = 0
        self.fail_on_call = fail_on_call
        self.batch_sizes = []

    def run(self, b, b_match, threshold):
        self.calls += 1
        if self.fail_on_call is not None and self.calls == self.fail_on_call:
            raise RuntimeError("injected backend failure")
        self.batch_sizes.append(len(b.reads))
        score = np.empty(b.n_jobs, np.float32)
        end = np.empty(b.n_jobs, np.int32)
        for t, ev in enumerate(b.chunks):
            for j in range(int(b.cand_off[t]), int(b.cand_off[t] + b.cand_cnt[t])):
                ro, rl, wo = int(b.r_off[j]), int(b.r_len[j]), int(b.row_off[j])
                init = None if b.first[j] else self.rows[wo:wo + rl].copy()
                c, e, row = oracle.dtw_f32(ev, self.r[ro:ro + rl], init_row=init, want_row=True)
                self.rows[wo:wo + rl] = row
                score[j], end[j] = c, e
        best, bs, mapped = oracle.decide(score, b.cand_off, b.cand_cnt, b.n_events, b_match, threshold)
        return score, end, best, bs, mapped
