"""fm_search_inexact_noalloc (workspace in the library's static device array) through the
C ABI: bit-identical to fm_search_inexact on consecutive calls, the second smaller than
the first, and on a third with the gapped search; the required hit total matches; a batch
whose workspace exceeds the array is refused on the host (FM_ERANGE)."""
import numpy as np
import pytest
import torch

import synth
from paper_1811_06127_amd import fm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def outputs(nreads, hit_cap):
    return (torch.full((max(hit_cap, 1), 4), -1, dtype=torch.int32, device="cuda"),
            torch.full((nreads + 1,), -1, dtype=torch.int64, device="cuda"),
            torch.full((max(nreads, 1),), -1, dtype=torch.int32, device="cuda"),
            torch.full((1,), -1, dtype=torch.int64, device="cuda"))


def compare(idx, rd, flags, zmax, hit_cap, tag):
    cd, od, zd = fm.reads_to_device(rd.codes, rd.offs, rd.z)
    need = fm.fm_search_inexact_workspace(idx, rd.count, int(rd.offs[-1]), flags, zmax, hit_cap)
    assert need <= fm.FM_NOALLOC_WS_BYTES
    want = fm.fm_search_inexact(idx, cd, od, zd, flags, zmax, hit_cap)
    wh, wo, ws = fm.hits_to_numpy(want, rd.count)
    hits, hoffs, status, req = outputs(rd.count, hit_cap)
    fm.fm_search_inexact_noalloc(idx, cd, od, zd, flags, zmax, hits, hoffs, status, req)
    torch.cuda.synchronize()
    go = hoffs.cpu().numpy().view(np.uint64)
    assert np.array_equal(go, wo), tag
    gh = hits[:int(go[-1])].cpu().numpy().view(np.uint32).reshape(-1, 4).copy().view(fm.HIT_DTYPE).reshape(-1)
    assert np.array_equal(gh, wh), tag
    assert np.array_equal(status[:rd.count].cpu().numpy().view(np.uint32), ws), tag
    assert int(req.item()) == want.required(), tag
    say(tag, "reads", rd.count, "hits", wh.size, "workspace", need, "ok")
    return wh.size


def test_noalloc_equals_workspace_call():
    R = synth.reference_with_repeats(400_000, 881, copy_frac=0.08, copy_len=(300, 2000), copy_sub=0.02,
                                     tandem_frac=0.01)
    idx = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_REVERSE)
    big = synth.simulate_reads(R, 40_000, 12, length=(50, 150), sub=(0.0, 0.03), z=(0, 2))
    small = synth.simulate_reads(R, 3_000, 13, length=(30, 90), sub=(0.0, 0.05), z=(0, 2))
    flags = fm.FM_BOTH | fm.FM_DARRAY
    assert compare(idx, big, flags, 2, 1 << 19, "first call") > 0
    assert compare(idx, small, flags, 2, 1 << 16, "second call, smaller") > 0
    compare(idx, small, flags | fm.FM_GAPS, 2, 1 << 17, "third call, gapped")
    # a batch whose workspace exceeds the static array is refused before any launch
    n = 400_000
    assert fm.fm_search_inexact_workspace(idx, n, n * 100, flags, 2, 1 << 20) > fm.FM_NOALLOC_WS_BYTES
    codes = torch.zeros(n * 100, dtype=torch.uint8, device="cuda")
    offs = torch.arange(0, n * 100 + 1, 100, dtype=torch.int64, device="cuda")
    z = torch.zeros(n, dtype=torch.uint8, device="cuda")
    hits, hoffs, status, req = outputs(n, 1 << 20)
    with pytest.raises(fm.FmError) as e:
        fm.fm_search_inexact_noalloc(idx, codes, offs, z, flags, 2, hits, hoffs, status, req)
    assert e.value.status == fm.FM_ERANGE
    assert int(hoffs[0].item()) == -1                   # nothing was written
    with pytest.raises(fm.FmError) as e:
        fm.fm_search_inexact_noalloc(idx, codes[:100], offs[:2], z[:1], flags | fm.FM_STATS, 2, hits, hoffs,
                                     status, req)
    assert e.value.status == fm.FM_EINVAL
    idx.free()
