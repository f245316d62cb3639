"""Locating (fm_locate, Eq. 4-5): the text position of every row of SA intervals, from
the SA values of every 32nd row and Psi^-1 walks, equals the oracle's suffix array."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1811_06127_amd import fm

pytestmark = pytest.mark.gpu

LAYOUTS = (64, 96, 128, 192, 224, 256, 448)


def say(*a):
    print(*a, flush=True)


def intervals(pairs):
    return torch.from_numpy(np.asarray(pairs, dtype=np.int64).astype(np.uint32).view(np.int32).reshape(-1, 2)).cuda()


def locate(idx, kl, cap=None):
    offs, pos = fm.fm_locate(idx, kl, cap)
    torch.cuda.synchronize()
    return offs.cpu().numpy(), pos.cpu().numpy().view(np.uint32)


def test_fig1_suffix_array():
    """R = ACAG: SA = 4 0 2 1 3 (Fig. 1); every row located one by one and as one interval."""
    R = np.array([0, 1, 0, 2], np.uint8)
    for flags in (fm.FM_LOAD_LOCATE, fm.FM_LOAD_LOCATE | fm.FM_LOAD_DEVICE_SORT):
        idx = fm.Index.from_text(R, occ_interval=64, flags=flags)
        assert idx.info()["sa_sample"] == 32
        offs, pos = locate(idx, intervals([(k, k) for k in range(5)] + [(0, 4)]))
        assert pos.tolist() == [4, 0, 2, 1, 3, 4, 0, 2, 1, 3]
        assert offs.tolist() == [0, 1, 2, 3, 4, 5, 10]
        idx.free()


@pytest.fixture(scope="module")
def text():
    R = synth.reference_with_repeats(70_001, 4243, copy_frac=0.08, copy_len=(300, 2000), copy_sub=0.02,
                                     tandem_frac=0.02, tandem_unit=(2, 12), tandem_len=(100, 400))
    return R, oracle.OracleIndex(R)


@pytest.mark.parametrize("device_sort", [False, True])
def test_every_row_all_layouts(text, device_sort):
    R, x = text
    n = R.size
    flags = fm.FM_LOAD_LOCATE | fm.FM_LOAD_ALL_LAYOUTS | (fm.FM_LOAD_DEVICE_SORT if device_sort else 0)
    idx = fm.Index.from_text(R, occ_interval=128, flags=flags)
    sa = x.sa
    rng = np.random.default_rng(3)
    # single rows, the whole range, misses, rows past the index and random ranges
    pairs = [(k, k) for k in range(n + 1)] + [(0, n), (1, 0), (n + 3, n + 9), (n, n + 1)]
    for _ in range(300):
        a = int(rng.integers(0, n + 1))
        pairs.append((a, min(n, a + int(rng.integers(0, 40)))))
    kl = intervals(pairs)
    want = []
    for k, l in pairs:
        if k <= l <= n:
            want.append(sa[k:l + 1])
    want = np.concatenate(want)
    for I in LAYOUTS:
        for waves, depth in ((4, 1), (16, 1), (0, 1), (8, 2), (16, 4), (4, 4)):
            idx.set_tuning(fm.FM_OP_LOCATE, occ_interval=I, waves_per_cu=waves, depth=depth)
            offs, pos = locate(idx, kl)
            assert offs[-1] == want.size and np.array_equal(pos, want), (I, waves, depth)
    assert idx.get_tuning(fm.FM_OP_EXACT)["occ_interval"] == 128   # locating has settings of its own
    with pytest.raises(fm.FmError):
        idx.set_tuning(fm.FM_OP_LOCATE, depth=3)
    with pytest.raises(fm.FmError):
        idx.set_tuning(fm.FM_OP_EXACT, depth=4)                     # four rows in flight: locating only
    # a capped call locates the first rows only and still reports the total, at every depth
    for depth in (1, 2, 4):
        idx.set_tuning(fm.FM_OP_LOCATE, occ_interval=128, waves_per_cu=16, depth=depth)
        offs, pos = locate(idx, kl, cap=1000)
        assert offs[-1] == want.size and np.array_equal(pos[:1000], want[:1000]), depth
        # fewer rows than lanes in flight
        offs, pos = locate(idx, kl, cap=7)
        assert np.array_equal(pos[:7], want[:7]), depth
    idx.free()


def test_hit_records_are_located_at_matching_windows(text):
    """The rows of inexact hits (fm_hit records, stride 4) sit at text windows within the
    hit's Hamming distance of the strand pattern."""
    R, x = text
    idx = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_LOCATE | fm.FM_LOAD_REVERSE)
    rd = synth.simulate_reads(R, 800, 17, length=(40, 90), sub=(0.0, 0.04), z=(0, 2))
    cd, od, zd = fm.reads_to_device(rd.codes, rd.offs, rd.z)
    bufs = fm.fm_search_inexact(idx, cd, od, zd, fm.FM_BOTH | fm.FM_DARRAY, 2, 1 << 16)
    hits, hoffs, status = fm.hits_to_numpy(bufs, rd.count)
    assert (status == fm.FM_OK).all()
    nh = int(hoffs[-1])
    offs, pos = locate(idx, bufs.hits[:nh])
    assert offs[-1] == int((hits["l"] - hits["k"] + 1).sum())
    sa = x.sa
    for h in range(nh):
        rows = np.arange(hits["k"][h], hits["l"][h] + 1)
        got = pos[offs[h]:offs[h + 1]]
        assert np.array_equal(got, sa[rows]), h
        r = int(hits["read"][h])
        W = oracle.strand_pattern(rd.read(r), int(hits["strand"][h]))
        for p in got:
            win = R[p:p + W.size]
            assert win.size == W.size and int((win != W).sum()) == int(hits["nmm"][h])
    say("located", offs[-1], "rows of", nh, "hits")
    idx.free()


def test_index_without_samples_is_rejected(text):
    R, _ = text
    idx = fm.Index.from_text(R[:5000], occ_interval=64)
    assert idx.info()["sa_sample"] == 0
    with pytest.raises(fm.FmError):
        fm.fm_locate(idx, intervals([(0, 3)]))
    idx.free()
