"""fm_probe_random_reads, the diagnostic that measures how fast the device serves
independent reads of random 32-byte blocks (one Occ8 bucket at I=64): argument checks,
the number of reads it reports, and a rate within the device's reach."""
import numpy as np
import pytest
import torch

import synth
from paper_1811_06127_amd import fm

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def idx():
    R = synth.iid_reference(50_000, 91)
    index = fm.Index.from_text(R, device=0, occ_interval=64)
    yield index
    index.free()


def test_reads_reported_and_sink_untouched(idx):
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    buf = torch.zeros(1 << 24, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    for span, rounds in ((4096, 1), (1 << 20, 3), (1 << 24, 16)):
        n = fm.probe_random_reads(idx, buf, span, rounds, sink)
        torch.cuda.synchronize()
        assert n == cus * 16 * 64 * rounds * 4, (span, rounds, n)
    # the buffer holds zeros, so no lane's sum equals the constant that writes the sink
    assert int(sink.item()) == 0


def test_rate_is_plausible(idx):
    buf = torch.zeros(1 << 28, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    fm.probe_random_reads(idx, buf, 1 << 28, 16, sink)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    n = fm.probe_random_reads(idx, buf, 1 << 28, 16, sink)
    ev[1].record()
    torch.cuda.synchronize()
    rate = n / (ev[0].elapsed_time(ev[1]) / 1e3)
    print("random 32-byte reads over 256 MiB: %.1fG/s" % (rate / 1e9))
    # every read moves at least 32 bytes, so the rate cannot exceed the memory bandwidth
    # over 32 B by much (the L2 serves a few), and a working launch is far above 1G/s
    assert 1e9 < rate < 8e12 / 32 * 1.5


@pytest.mark.parametrize("span,rounds,offset", [(3000, 1, 0), (4096 + 32, 1, 0), (2048, 1, 0), (4096, 0, 0),
                                                 (4096, 5000, 0), (4096, 1, 4)])
def test_bad_arguments(idx, span, rounds, offset):
    buf = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    n = fm.C.c_uint64(0)
    st = fm.lib().fm_probe_random_reads(idx.handle, buf.data_ptr() + offset, span, rounds, sink.data_ptr(),
                                        fm.C.byref(n), None)
    assert st == fm.FM_EINVAL
    assert n.value == 0
