"""Launch graphs (fm_plan_*): every replay equals the eager call on whatever the captured
buffers hold at replay time, with unrelated eager work and synchronisations between
replays."""
import numpy as np
import pytest
import torch

import synth
from paper_1811_06127_amd import fm

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


def eager(idx, rd, flags, zmax):
    codes, offs, z = fm.reads_to_device(rd.codes, rd.offs, rd.z)
    n = rd.count
    ex = fm.fm_search_exact(idx, codes, offs, fm.FM_BOTH)
    bufs = fm.fm_search_inexact(idx, codes, offs, z, flags, zmax, 8 * n)
    torch.cuda.synchronize()
    return ex.cpu().numpy().copy(), fm.hits_to_numpy(bufs, n)


@pytest.mark.parametrize("use_d", [True, False])
def test_plan_replays_match_eager(use_d):
    R = synth.reference_with_repeats(120_001, 515, copy_frac=0.06, copy_len=(300, 2000), copy_sub=0.02)
    idx = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_REVERSE)
    flags = fm.FM_BOTH | (fm.FM_DARRAY if use_d else 0)
    # equal read lengths, so every batch has the captured shape
    batches = [synth.simulate_reads(R, 700, s, length=(90, 90), sub=(0.0, 0.03), z=(0, 2)) for s in (61, 62, 63)]
    want = [eager(idx, rd, flags, 2) for rd in batches]
    n = batches[0].count
    codes, offs, z = fm.reads_to_device(batches[0].codes, batches[0].offs, batches[0].z)
    ex_out = torch.empty((2 * n, 2), dtype=torch.int32, device="cuda")
    ex_ws = torch.zeros(fm.fm_search_exact_workspace(idx, n, fm.FM_BOTH), dtype=torch.uint8, device="cuda")
    bufs = fm.InexactBuffers(idx, n, int(batches[0].offs[-1]), flags, 2, 8 * n, "cuda")
    plans = [fm.Plan(idx, fm.FM_OP_EXACT, codes, offs, None, fm.FM_BOTH, out=ex_out, ws=ex_ws),
             fm.Plan(idx, fm.FM_OP_INEXACT, codes, offs, z, flags, 2, bufs=bufs)]
    other = synth.simulate_reads(R, 333, 64, length=(40, 160), sub=(0.0, 0.03), z=(0, 2))
    for rep, b in enumerate([0, 1, 0, 2, 2]):
        rd = batches[b]
        codes.copy_(torch.from_numpy(rd.codes))
        z.copy_(torch.from_numpy(rd.z))
        for p in plans:
            p.launch()
        torch.cuda.synchronize()
        got_ex = ex_out.cpu().numpy()
        got_in = fm.hits_to_numpy(bufs, n)
        say("replay", rep, "batch", b, "hits", int(got_in[1][-1]))
        assert np.array_equal(got_ex, want[b][0]), (rep, b)
        assert all(np.array_equal(x, y) for x, y in zip(got_in, want[b][1])), (rep, b)
        # unrelated eager work between replays
        eager(idx, other, flags, 2)
    for p in plans:
        p.free()


def test_fused_plan_replays_match_eager():
    """A plan of fm_search_both replays to the eager results of the separate calls."""
    R = synth.reference_with_repeats(120_001, 516, copy_frac=0.06, copy_len=(300, 2000), copy_sub=0.02)
    idx = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_REVERSE)
    flags = fm.FM_BOTH | fm.FM_DARRAY
    batches = [synth.simulate_reads(R, 600, s, length=(80, 80), sub=(0.0, 0.03), z=(0, 2)) for s in (71, 72)]
    want = [eager(idx, rd, flags, 2) for rd in batches]
    n = batches[0].count
    codes, offs, z = fm.reads_to_device(batches[0].codes, batches[0].offs, batches[0].z)
    ex_out = torch.empty((2 * n, 2), dtype=torch.int32, device="cuda")
    bufs = fm.InexactBuffers(idx, n, int(batches[0].offs[-1]), flags, 2, 8 * n, "cuda")
    plan = fm.Plan.both(idx, codes, offs, z, fm.FM_BOTH, flags, 2, ex_out, bufs)
    other = synth.simulate_reads(R, 200, 73, length=(40, 160), sub=(0.0, 0.03), z=(0, 2))
    for rep, b in enumerate([0, 1, 1, 0]):
        rd = batches[b]
        codes.copy_(torch.from_numpy(rd.codes))
        z.copy_(torch.from_numpy(rd.z))
        plan.launch()
        torch.cuda.synchronize()
        assert np.array_equal(ex_out.cpu().numpy(), want[b][0]), (rep, b)
        assert all(np.array_equal(x, y) for x, y in zip(fm.hits_to_numpy(bufs, n), want[b][1])), (rep, b)
        eager(idx, other, flags, 2)
    plan.free()


def test_timed_plans_record_phases_and_match_eager():
    """Plans created while phase timing is on are captured one graph per phase, with HIP
    events recorded between them on the replay stream: every replay still equals the eager
    call, fm_plan_phase_times gives positive times of the last replay whose sum is within
    the replay's event-timed span, and an untimed plan refuses the call."""
    R = synth.reference_with_repeats(120_001, 517, copy_frac=0.06, copy_len=(300, 2000), copy_sub=0.02)
    idx = fm.Index.from_text(R, occ_interval=64, flags=fm.FM_LOAD_REVERSE)
    flags = fm.FM_BOTH | fm.FM_DARRAY
    batches = [synth.simulate_reads(R, 2000, s, length=(100, 100), sub=(0.0, 0.03), z=(0, 2)) for s in (81, 82)]
    want = [eager(idx, rd, flags, 2) for rd in batches]
    n = batches[0].count
    codes, offs, z = fm.reads_to_device(batches[0].codes, batches[0].offs, batches[0].z)
    ex_out = torch.empty((2 * n, 2), dtype=torch.int32, device="cuda")
    ex_ws = torch.zeros(fm.fm_search_exact_workspace(idx, n, fm.FM_BOTH), dtype=torch.uint8, device="cuda")
    bufs = fm.InexactBuffers(idx, n, int(batches[0].offs[-1]), flags, 2, 8 * n, "cuda")
    idx.phase_timing(4)
    both = fm.Plan.both(idx, codes, offs, z, fm.FM_BOTH, flags, 2, ex_out, bufs)
    exact = fm.Plan(idx, fm.FM_OP_EXACT, codes, offs, None, fm.FM_BOTH, out=ex_out, ws=ex_ws)
    idx.phase_timing(0)
    untimed = fm.Plan.both(idx, codes, offs, z, fm.FM_BOTH, flags, 2, ex_out, bufs)
    with pytest.raises(fm.FmError):
        untimed.phase_times()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    for rep, b in enumerate([0, 1, 1, 0]):
        rd = batches[b]
        codes.copy_(torch.from_numpy(rd.codes))
        z.copy_(torch.from_numpy(rd.z))
        plan = untimed if rep == 2 else both
        ev[0].record()
        plan.launch()
        ev[1].record()
        torch.cuda.synchronize()
        assert np.array_equal(ex_out.cpu().numpy(), want[b][0]), (rep, b)
        assert all(np.array_equal(x, y) for x, y in zip(fm.hits_to_numpy(bufs, n), want[b][1])), (rep, b)
        if plan is both:
            ph = both.phase_times()
            span = ev[0].elapsed_time(ev[1])
            say("replay", rep, "phases", ph, "span %.3f ms" % span)
            assert ph["d_walk"] > 0 and ph["dfs"] > 0 and ph["compaction"] > 0 and ph["exact_walk"] == 0
            assert ph["d_walk"] + ph["dfs"] + ph["compaction"] <= span * 1.01 + 0.01
        exact.launch()
        torch.cuda.synchronize()
        assert np.array_equal(ex_out.cpu().numpy(), want[b][0]), ("exact", rep, b)
        assert exact.phase_times()["exact_walk"] > 0
    for p in (both, exact, untimed):
        p.free()
