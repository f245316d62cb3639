"""Host-side pieces of bench.py, on the CPU: the search's own Occ8 query set (the third
micro-benchmark set) expands exactly the nodes of Listing 2's substitution search with the
D bound, checked against the oracle's node count with the oracle's Occ and D standing in
for fm_occ8 and fm_darray."""
import types

import numpy as np

import bench
import oracle
import synth


class _Host:
    """An array standing in for a device tensor: .cpu().numpy() and .to(dev) return it."""

    def __init__(self, a):
        self.a = a

    def cpu(self):
        return self

    def numpy(self):
        return self.a

    def to(self, dev):
        return self.a


def test_search_trace_expands_the_oracle_nodes():
    R = synth.reference_with_repeats(50_003, 4245, copy_frac=0.08, copy_len=(300, 2000), copy_sub=0.02)
    x = oracle.OracleIndex(R)
    xr = oracle.OracleIndex(oracle.reverse_text(R))
    rd = synth.simulate_reads(R, 400, 46, length=(60, 60), sub=(0.0, 0.03), z=(0, 2))
    fm = types.SimpleNamespace(
        FM_BOTH=3,
        reads_to_device=lambda c, o, z, dev: (c, o, z),
        fm_darray=lambda idx, c, o, total, flags: _Host(xr.darray(c, o, oracle.BOTH)),
        fm_occ8=lambda idx, q: _Host(x.occ8(q.view(np.uint32)).view(np.int32)))
    torch = types.SimpleNamespace(from_numpy=_Host)
    idx = types.SimpleNamespace(info=lambda: {"C": [int(v) for v in x.C], "n": int(R.size)})
    trace, _ = bench.search_trace(fm, torch, idx, rd, rd.count, None)
    _, _, nodes = x.inexact(rd.codes, rd.offs, rd.z, oracle.BOTH, "listing2_darray", rev=xr, return_nodes=True)
    assert trace.shape == (int(nodes.sum()), 2)
    # every query is a valid interval as the kernels issue it: 1 <= k <= l + 1, l <= n
    assert (trace[:, 0] >= 1).all() and (trace[:, 1] <= R.size).all() and (trace[:, 0] <= trace[:, 1] + 1).all()
