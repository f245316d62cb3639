"""Index construction on the device (fm_bwt_device, FM_LOAD_DEVICE_SORT): the BWT equals
the oracle's (suffixes sorted by direct comparison) and the host builder's, and an index
built either way answers searches identically."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1811_06127_amd import fm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def texts():
    rng = np.random.default_rng(12)
    yield "empty", np.zeros(0, np.uint8)
    yield "one symbol", np.array([2], np.uint8)
    yield "run of A", np.zeros(5000, np.uint8)
    yield "run of T", np.full(777, 3, np.uint8)
    yield "period 2", np.tile(np.array([0, 1], np.uint8), 3000)
    yield "period 7", np.tile(rng.integers(0, 4, 7).astype(np.uint8), 1000)
    yield "short", rng.integers(0, 4, 20).astype(np.uint8)
    yield "repeats", synth.reference_with_repeats(70_001, 4242, copy_frac=0.08, copy_len=(300, 2000), copy_sub=0.02,
                                                  tandem_frac=0.02, tandem_unit=(2, 12), tandem_len=(100, 400))


@pytest.mark.parametrize("name,R", list(texts()), ids=[t[0] for t in texts()])
def test_device_bwt_equals_oracle_and_host(name, R):
    say("text", name, R.size)
    got, dr = fm.fm_bwt_device(R)
    host, hdr = fm.fm_bwt_host(R)
    assert dr == hdr and np.array_equal(got, host)
    if R.size <= 80_000:
        x = oracle.OracleIndex(R)
        assert dr == x.dollar_row
        want = x.bwt.copy()
        assert np.array_equal(got, want)
    rev, rdr = fm.fm_bwt_device(oracle.reverse_text(R))
    hrev, hrdr = fm.fm_bwt_host(oracle.reverse_text(R))
    assert rdr == hrdr and np.array_equal(rev, hrev)


def test_device_bwt_large_text_with_copies():
    """2^22 bases with 5% diverged copies: equal to the host builder."""
    R = synth.reference_with_repeats(1 << 22, 77)
    got, dr = fm.fm_bwt_device(R)
    host, hdr = fm.fm_bwt_host(R)
    assert dr == hdr and np.array_equal(got, host)


def test_device_built_index_searches_alike():
    R = synth.reference_with_repeats(300_001, 91, copy_frac=0.08, tandem_frac=0.01)
    a = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_REVERSE)
    b = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_REVERSE | fm.FM_LOAD_DEVICE_SORT)
    assert a.info() == b.info()
    rd = synth.simulate_reads(R, 3000, 5, length=(30, 120), sub=(0.0, 0.03), z=(0, 2))
    cd, od, zd = fm.reads_to_device(rd.codes, rd.offs, rd.z)
    flags = fm.FM_BOTH | fm.FM_DARRAY
    ea, ba = fm.fm_search_both(a, cd, od, zd, fm.FM_BOTH, flags, 2, 1 << 16)
    ha = fm.hits_to_numpy(ba, rd.count)
    eb, bb = fm.fm_search_both(b, cd, od, zd, fm.FM_BOTH, flags, 2, 1 << 16)
    hb = fm.hits_to_numpy(bb, rd.count)
    assert torch.equal(ea, eb)
    for u, v in zip(ha, hb):
        assert np.array_equal(u, v)
    with pytest.raises(fm.FmError):
        fm.Index.from_text(np.array([0, 1, 5], np.uint8), flags=fm.FM_LOAD_DEVICE_SORT)
    a.free()
    b.free()
