"""Host-side checks of the C ABI: the library loads without a GPU, exports
every entry point the header declares, and rejects bad arguments before
touching the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    from paper_2310_05037_amd import lib
    if not os.path.exists(lib.LIB_PATH):
        from paper_2310_05037_amd import build
        build.build()
    return lib


def _declared():
    text = open(os.path.join(ROOT, "include", "rawalign.h")).read()
    return sorted(set(re.findall(r"^(?:int|const char \*)\s*(rawalign_\w+)\(", text, re.M)))


def test_header_declarations_are_exported(L):
    decl = _declared()
    assert len(decl) >= 10
    assert sorted(L.EXPORTS) == decl
    so = L.load()
    for name in decl:
        assert hasattr(so, name), name


def test_version_and_defaults(L):
    assert L.rawalign_version().startswith("rawalign-mi355x")
    o = L.opts_default()
    assert o.mode == L.MODE_PERSISTENT and o.streams == 1 and o.lo_waves_per_cu == 0


def test_argument_errors_without_device(L):
    so = L.load()
    vp = ctypes.c_void_p
    fake = vp(0x1000)
    # negative pair count
    rc = so.rawalign_dtw_batch(fake, 10, fake, fake, fake, 10, fake, fake, -1, fake, fake, None)
    assert rc == L.RAWALIGN_EINVAL and b"n_pairs" in so.rawalign_last_error()
    # null offsets
    rc = so.rawalign_dtw_batch(fake, 10, None, fake, fake, 10, fake, fake, 3, fake, fake, None)
    assert rc == L.RAWALIGN_EINVAL and b"null" in so.rawalign_last_error()
    # zero pairs: nothing to do, success
    rc = so.rawalign_dtw_batch(None, 0, None, None, None, 0, None, None, 0, None, None, None)
    assert rc == L.RAWALIGN_OK
    # bad option values
    o = L.opts_default()
    o.mode = 9
    rc = so.rawalign_dtw_batch_ex(fake, 10, fake, fake, fake, 10, fake, fake, 2, fake, fake, None, ctypes.byref(o))
    assert rc == L.RAWALIGN_EINVAL and b"mode" in so.rawalign_last_error()
    o = L.opts_default()
    o.streams = 2
    rc = so.rawalign_dtw_batch_ex(fake, 10, fake, fake, fake, 10, fake, fake, 2, fake, fake, None, ctypes.byref(o))
    assert rc == L.RAWALIGN_EINVAL and b"streams" in so.rawalign_last_error()
    o = L.opts_default()
    o.long_waves_per_cu = 99
    rc = so.rawalign_dtw_batch_ex(fake, 10, fake, fake, fake, 10, fake, fake, 2, fake, fake, None, ctypes.byref(o))
    assert rc == L.RAWALIGN_EINVAL and b"waves_per_cu" in so.rawalign_last_error()
    o = L.opts_default()
    o.long_kernel = 7
    rc = so.rawalign_dtw_batch_ex(fake, 10, fake, fake, fake, 10, fake, fake, 2, fake, fake, None, ctypes.byref(o))
    assert rc == L.RAWALIGN_EINVAL and b"long_kernel" in so.rawalign_last_error()
    with pytest.raises(ValueError):
        L.make_opts(pipe_wave=4)   # a misspelt field is an error, not a no-op
    # the anti-diagonal kernel runs plain batches only, not the streaming extension
    o = L.opts_default()
    o.long_kernel = L.LONG_ANTIDIAG
    rc = so.rawalign_dtw_extend(fake, 10, fake, fake, fake, 10, fake, fake, fake, 10, fake, fake, 2, fake, fake,
                                None, ctypes.byref(o))
    assert rc == L.RAWALIGN_EINVAL and b"long_kernel" in so.rawalign_last_error()
    # extend without a row arena
    rc = so.rawalign_dtw_extend(fake, 10, fake, fake, fake, 10, fake, fake, None, 0, fake, fake, 2, fake, fake,
                                None, None)
    assert rc == L.RAWALIGN_EINVAL
    # early termination: bad block size, negative max_query, missing rows
    def bnb(block_rows=512, max_query=100, rows=fake, n_reads=2):
        return so.rawalign_map_bnb(fake, 10, fake, fake, fake, 10, fake, fake, 2, fake, fake, fake, n_reads, 0.4,
                                   20.0, max_query, block_rows, rows, 10, fake, fake, fake, fake, fake, fake, None,
                                   None)
    assert bnb(block_rows=32) == L.RAWALIGN_EINVAL and b"block_rows" in so.rawalign_last_error()
    assert bnb(max_query=-1) == L.RAWALIGN_EINVAL and b"max_query" in so.rawalign_last_error()
    assert bnb(rows=None) == L.RAWALIGN_EINVAL and b"rows" in so.rawalign_last_error()
    assert bnb(n_reads=-1) == L.RAWALIGN_EINVAL and b"n_reads" in so.rawalign_last_error()
    # decide with a negative read count
    rc = so.rawalign_decide(fake, 1, fake, fake, fake, -1, 0.4, 20.0, fake, fake, fake, None)
    assert rc == L.RAWALIGN_EINVAL
    # global alignment: the end output is optional, the anti-diagonal kernel is not offered
    rc = so.rawalign_dtw_global_batch(None, 0, None, None, None, 0, None, None, 0, None, None, None, None)
    assert rc == L.RAWALIGN_OK
    rc = so.rawalign_dtw_global_batch(fake, 10, fake, fake, fake, 10, fake, fake, -1, fake, None, None, None)
    assert rc == L.RAWALIGN_EINVAL and b"n_pairs" in so.rawalign_last_error()
    rc = so.rawalign_dtw_global_batch(fake, 10, fake, fake, fake, 10, fake, fake, 2, None, None, None, None)
    assert rc == L.RAWALIGN_EINVAL and b"null" in so.rawalign_last_error()
    o = L.opts_default()
    o.long_kernel = L.LONG_ANTIDIAG
    rc = so.rawalign_dtw_global_batch(fake, 10, fake, fake, fake, 10, fake, fake, 2, fake, None, None,
                                      ctypes.byref(o))
    assert rc == L.RAWALIGN_EINVAL and b"long_kernel" in so.rawalign_last_error()
    # alignment start: out_start required, striped long kernel only, zero pairs is a no-op
    rc = so.rawalign_dtw_span(fake, 10, fake, fake, fake, 10, fake, fake, 2, fake, fake, None, None, None)
    assert rc == L.RAWALIGN_EINVAL and b"out_start" in so.rawalign_last_error()
    o = L.opts_default()
    o.long_kernel = L.LONG_ANTIDIAG
    rc = so.rawalign_dtw_span(fake, 10, fake, fake, fake, 10, fake, fake, 2, fake, fake, fake, None,
                              ctypes.byref(o))
    assert rc == L.RAWALIGN_EINVAL and b"long_kernel" in so.rawalign_last_error()
    rc = so.rawalign_dtw_span(None, 0, None, None, None, 0, None, None, 0, None, None, None, None, None)
    assert rc == L.RAWALIGN_OK
    rc = so.rawalign_dtw_span(fake, 10, fake, fake, fake, 10, fake, fake, -3, fake, fake, fake, None, None)
    assert rc == L.RAWALIGN_EINVAL and b"n_pairs" in so.rawalign_last_error()
    # chain sums and decision
    def chains(n_gaps=4, n_chains=2, n_reads=1, gap_cost=fake, events=fake, threshold=20.0):
        return so.rawalign_chain_decide(gap_cost, n_gaps, fake, fake, events, n_chains, fake, fake, n_reads, 0.4,
                                        threshold, fake, fake, fake, fake, None)
    assert chains(n_chains=-1) == L.RAWALIGN_EINVAL and b"n_chains" in so.rawalign_last_error()
    assert chains(events=None) == L.RAWALIGN_EINVAL and b"null" in so.rawalign_last_error()
    assert chains(gap_cost=None) == L.RAWALIGN_EINVAL and b"gap_cost" in so.rawalign_last_error()
    assert chains(threshold=float("nan")) == L.RAWALIGN_EINVAL
    assert chains(n_gaps=0, n_chains=0, n_reads=0) == L.RAWALIGN_OK
    # allocation-free batch: refused beyond its fixed scratch, before any device call
    big = L.RAWALIGN_NOALLOC_MAX_PAIRS + 1
    rc = so.rawalign_dtw_batch_noalloc(fake, 10, fake, fake, fake, 10, fake, fake, big, fake, fake, None)
    assert rc == L.RAWALIGN_EINVAL and b"exceeds" in so.rawalign_last_error()
    rc = so.rawalign_dtw_batch_noalloc(fake, 10, fake, fake, fake, 10, fake, fake, -1, fake, fake, None)
    assert rc == L.RAWALIGN_EINVAL and b"n_pairs" in so.rawalign_last_error()
    rc = so.rawalign_dtw_batch_noalloc(None, 0, None, None, None, 0, None, None, 0, None, None, None)
    assert rc == L.RAWALIGN_OK


def test_binding_rejects_host_tensors(L):
    import torch
    t = torch.zeros(4)
    with pytest.raises(TypeError):
        L._dev(t, torch.float32, "q")


def test_band_argument_errors_without_device(L):
    so = L.load()
    fake = ctypes.c_void_p(0x1000)
    # the band array is required, the end output too; zero pairs is a no-op
    rc = so.rawalign_dtw_band(fake, 10, fake, fake, fake, 10, fake, fake, None, 2, fake, fake, None)
    assert rc == L.RAWALIGN_EINVAL and b"band" in so.rawalign_last_error()
    rc = so.rawalign_dtw_band(fake, 10, fake, fake, fake, 10, fake, fake, fake, -1, fake, fake, None)
    assert rc == L.RAWALIGN_EINVAL and b"n_pairs" in so.rawalign_last_error()
    rc = so.rawalign_dtw_band(fake, 10, None, fake, fake, 10, fake, fake, fake, 2, fake, fake, None)
    assert rc == L.RAWALIGN_EINVAL and b"null" in so.rawalign_last_error()
    rc = so.rawalign_dtw_band(None, 0, None, None, None, 0, None, None, None, 0, None, None, None)
    assert rc == L.RAWALIGN_OK


def test_path_argument_errors_without_device(L):
    so = L.load()
    fake = ctypes.c_void_p(0x1000)

    def path(dir_off=fake, dirs=fake, dir_size=100, path_off=fake, path_size=10, n_pairs=2, out_start=fake):
        return so.rawalign_dtw_path(fake, 10, fake, fake, fake, 10, fake, fake, n_pairs, dir_off, dirs, dir_size,
                                    path_off, fake, fake, path_size, fake, fake, out_start, None, None)
    assert path(dir_size=-1) == L.RAWALIGN_EINVAL and b"dir_size" in so.rawalign_last_error()
    assert path(path_size=-1) == L.RAWALIGN_EINVAL and b"path_size" in so.rawalign_last_error()
    assert path(path_off=None) == L.RAWALIGN_EINVAL and b"path_off" in so.rawalign_last_error()
    assert path(dir_off=None) == L.RAWALIGN_EINVAL and b"dir_off" in so.rawalign_last_error()
    assert path(dirs=None) == L.RAWALIGN_EINVAL and b"dirs" in so.rawalign_last_error()
    assert path(out_start=None) == L.RAWALIGN_EINVAL and b"out_start" in so.rawalign_last_error()
    assert path(n_pairs=-1) == L.RAWALIGN_EINVAL and b"n_pairs" in so.rawalign_last_error()
    assert path(n_pairs=0, path_off=None, dir_off=None) == L.RAWALIGN_OK


def test_path_workspace_sizes(L):
    """n * (64 * ceil(m / 2048) + 1) words per pair, packed in order."""
    import numpy as np
    off, words = L.path_workspace(np.array([3, 0, 5]), np.array([2048, 10, 2049]))
    assert list(off) == [0, 3 * 65, 3 * 65] and words == 3 * 65 + 5 * 129
