"""The request server: each request's result is byte-identical whether it is served
alone or batched with others, equals a direct search call, and matches the oracle."""
import threading
import time

import numpy as np
import pytest

import oracle
import synth
from paper_1811_06127_amd import fm

pytestmark = pytest.mark.gpu

FLAGS = fm.FM_BOTH | fm.FM_DARRAY


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def setup():
    R = synth.reference_with_repeats(200_003, 777, copy_frac=0.06, copy_len=(300, 3000), copy_sub=0.02,
                                     tandem_frac=0.01, tandem_unit=(2, 30), tandem_len=(100, 500))
    idx = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_REVERSE)
    reqs = synth.request_stream(R, 40, 2000.0, seed=3100, size=(1, 1500), length=(50, 250),
                                sub=(0.005, 0.03), z=(0, 2))
    say("index and", len(reqs), "requests,", sum(r.reads.count for r in reqs), "reads")
    return R, idx, reqs


def same(a, b):
    return (a.error == b.error and np.array_equal(a.status, b.status) and np.array_equal(a.hit_offs, b.hit_offs)
            and a.hits.tobytes() == b.hits.tobytes())


def serve_alone(idx, reqs, **kw):
    out = []
    with fm.Server(idx, **kw) as s:
        for r in reqs:
            t = s.submit(r.reads.codes, r.reads.offs, r.reads.z)
            out.append(s.wait(t))
            s.release(t)
        st = s.stats()
    return out, st


def serve_mixed(idx, reqs, **kw):
    """All requests submitted from one thread with short gaps while another waits."""
    with fm.Server(idx, **kw) as s:
        tickets = []

        def producer():
            for r in reqs:
                tickets.append(s.submit(r.reads.codes, r.reads.offs, r.reads.z))
                time.sleep(0.0002)

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        out = []
        for t in tickets:
            out.append(s.wait(t, timeout=60.0))
            s.release(t)
        st = s.stats()
    return out, st


def test_alone_equals_mixed_equals_direct(setup):
    R, idx, reqs = setup
    alone, st_a = serve_alone(idx, reqs, lanes=2, flags=FLAGS, zmax=2, arena_bytes=256 << 20)
    say("alone", st_a)
    mixed, st_m = serve_mixed(idx, reqs, lanes=3, flags=FLAGS, zmax=2, arena_bytes=256 << 20)
    say("mixed", st_m)
    assert st_a["batches"] == len(reqs) and st_a["error"] == 0 and st_m["error"] == 0
    assert st_m["requests_done"] == len(reqs)
    # batching happened: some batch held several requests
    assert len({m.batch for m in mixed}) < len(reqs)
    for r, a, m in zip(reqs, alone, mixed):
        assert a is not None and m is not None
        assert a.error == fm.FM_OK and (a.status == fm.FM_OK).all()
        assert same(a, m), r.rid
        assert a.t_submit <= a.t_launch <= a.t_done
    # equal to a direct call of the search on the request alone
    for r, a in zip(reqs[:10], alone[:10]):
        cd, od, zd = fm.reads_to_device(r.reads.codes, r.reads.offs, r.reads.z)
        bufs = fm.fm_search_inexact(idx, cd, od, zd, FLAGS, 2, 1 << 20)
        hits, hoffs, status = fm.hits_to_numpy(bufs, r.reads.count)
        assert np.array_equal(hoffs, a.hit_offs) and np.array_equal(status, a.status)
        assert hits.tobytes() == a.hits.tobytes()


def test_matches_oracle(setup):
    R, idx, reqs = setup
    x = oracle.OracleIndex(R)
    xr = oracle.OracleIndex(oracle.reverse_text(R))
    picked = [r for r in reqs if r.reads.count <= 300][:4]
    got, _ = serve_mixed(idx, picked, lanes=2, flags=FLAGS, zmax=2, arena_bytes=64 << 20)
    for r, g in zip(picked, got):
        wh, wo = x.inexact(r.reads.codes, r.reads.offs, r.reads.z, oracle.BOTH, "listing2_darray", rev=xr)
        assert np.array_equal(g.hit_offs, wo)
        for f in ("read", "k", "l", "strand"):
            assert np.array_equal(g.hits[f], wh[f]), f
        assert np.array_equal(g.hits["nmm"], wh["d"])


def test_hit_overflow_retry_and_limits(setup):
    R, idx, reqs = setup
    base, _ = serve_alone(idx, reqs[:8], lanes=1, flags=FLAGS, zmax=2, arena_bytes=128 << 20)
    # no hit reserve: every batch with hits is searched again with room for them
    got, st = serve_mixed(idx, reqs[:8], lanes=2, flags=FLAGS, zmax=2, hit_reserve=0, arena_bytes=128 << 20)
    assert st["retries"] > 0
    for a, b in zip(base, got):
        assert same(a, b)
    # a tiny arena: the retry moves the batch to larger buffers of its own
    small = [r for r in reqs if 100 <= r.reads.count <= 300][:3]
    base, _ = serve_alone(idx, small, lanes=1, flags=FLAGS, zmax=2, arena_bytes=64 << 20)
    need = max(fm.fm_server_bytes(fm.server_opts(flags=FLAGS, zmax=2, hit_reserve=0), r.reads.count,
                                  int(r.reads.offs[-1])) for r in small)
    got, st = serve_alone(idx, small, lanes=1, flags=FLAGS, zmax=2, hit_reserve=0, arena_bytes=need + 256)
    assert st["retries"] > 0
    for a, b in zip(base, got):
        assert same(a, b)
    # a request that cannot fit a lane is refused at submission
    with fm.Server(idx, lanes=2, flags=FLAGS, zmax=2, arena_bytes=1 << 16) as s:
        big = max(reqs, key=lambda r: r.reads.count)
        with pytest.raises(fm.FmError) as e:
            s.submit(big.reads.codes, big.reads.offs, big.reads.z)
        assert e.value.status == fm.FM_ERANGE
        # an empty request completes with no hits
        t = s.submit(np.zeros(0, np.uint8), np.zeros(1, np.uint64), np.zeros(0, np.uint8))
        r = s.wait(t, timeout=30.0)
        assert r is not None and r.hits.size == 0 and r.hit_offs.tolist() == [0]


def test_small_ring_backpressure(setup):
    """A ring that holds about two requests' symbols: submissions wait for uploads, and
    every result still equals the request served alone."""
    R, idx, reqs = setup
    sub = reqs[:16]
    base, _ = serve_alone(idx, sub, lanes=2, flags=FLAGS, zmax=2, arena_bytes=256 << 20)
    biggest = max(int(r.reads.offs[-1]) for r in sub)
    got, st = serve_mixed(idx, sub, lanes=2, flags=FLAGS, zmax=2, arena_bytes=256 << 20, ring_bytes=2 * biggest + 64)
    assert st["requests_done"] == len(sub) and st["error"] == 0
    for a, b in zip(base, got):
        assert same(a, b)
        assert b.t_submit <= b.t_launch <= b.t_done
