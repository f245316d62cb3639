"""The seeded generators are deterministic and produce the stated shapes (no GPU)."""
import numpy as np

import synth


def test_splitmix64_published_vector():
    # First outputs of SplitMix64 seeded with 0 (the generator's reference sequence).
    got = synth.splitmix64(0, np.arange(3, dtype=np.uint64)).tolist()
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_reference_with_repeats_shape_and_determinism():
    a = synth.reference_with_repeats(200_000, 5, copy_frac=0.05, copy_len=(500, 5000), tandem_frac=0.01)
    b = synth.reference_with_repeats(200_000, 5, copy_frac=0.05, copy_len=(500, 5000), tandem_frac=0.01)
    assert a.size == 200_000 and a.dtype == np.uint8 and a.max() <= 3
    assert np.array_equal(a, b)
    counts = np.bincount(a, minlength=4) / a.size
    assert np.all(np.abs(counts - 0.25) < 0.01)


def test_simulated_reads_come_from_the_text():
    ref = synth.iid_reference(50_000, 9)
    rd = synth.simulate_reads(ref, 500, 10, length=(50, 250), sub=(0.0, 0.0), z=(0, 2))
    assert rd.count == 500 and rd.offs[-1] == rd.codes.size
    for r in range(0, 500, 37):
        w = rd.read(r)
        p = int(rd.pos[r])
        seg = ref[p:p + w.size]
        if rd.strand[r]:
            seg = 3 - seg[::-1]
        assert np.array_equal(w, seg)
    assert set(np.unique(rd.z)) <= {0, 1, 2}


def test_small_exact_workload():
    w = synth.small_exact_workload()
    assert w.ref.size == 65536 and w.reads.count == 10_000
    assert np.all(np.diff(w.reads.offs.astype(np.int64)) == 32)
    p = int(w.reads.pos[3])
    assert np.array_equal(w.reads.read(3), w.ref[p:p + 32])


def test_occ8_queries_ranges():
    q = synth.occ8_queries(1000, 10_000, 4, "uniform")
    assert q[:, 0].max() <= 1001 and q[:, 1].max() <= 1000
    q = synth.occ8_queries(1000, 10_000, 4, "narrow")
    assert np.all(q[:, 0].astype(np.int64) <= q[:, 1].astype(np.int64) + 1)


def test_stream_helpers_and_threaded_blocks():
    """Exponential gaps, forked streams and the block-threaded bases draw the same values
    as one sequential stream."""
    r = synth.Rng(77)
    g = r.exponential(2.0, 200_000)
    assert (g > 0).all() and abs(g.mean() - 0.5) < 0.01
    a, b = synth.Rng(9), synth.Rng(9)
    f = a.fork(1000)
    assert a.ctr == 1000 and np.array_equal(f.u64(1000), b.u64(1000))
    n = (1 << 20) * 32 * 3 + 17                      # several blocks and a ragged tail
    x = synth.Rng(5).bases(n)
    w = synth.Rng(5).u64((n + 31) // 32)
    assert np.array_equal(x[:64], ((w[:2, None] >> np.arange(0, 64, 2, dtype=np.uint64)) & np.uint64(3)).reshape(-1))
    assert np.array_equal(x[-17:], ((w[-1] >> np.arange(0, 34, 2, dtype=np.uint64)) & np.uint64(3)).astype(np.uint8))
    ref = synth.reference_families(300_000, 4)
    assert np.array_equal(ref, synth.reference_families(300_000, 4)) and ref.size == 300_000
