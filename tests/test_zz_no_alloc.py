"""qh_phase_noalloc, the entry point for callers that cannot allocate device memory,
called through the C ABI: its outputs equal qh_phase's bit for bit, on two calls in a row
(the second with a smaller graph, so the counters it finds are the first call's), for SNP
graphs (the parity round, whose per-component counters live in the library's static
device array) and read graphs (the vote, which needs no scratch)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2603_25762_amd as qh
import synth
from gpu_helpers import cpu, gpu_graph

pytestmark = pytest.mark.gpu


def _spins(n, seed):
    rng = np.random.default_rng(seed)
    return qh.to_device(np.where(rng.random(n) < 0.5, 1, -1).astype(np.int8))


@pytest.mark.parametrize("kind", ["snp_llr", "read_signed"])
def test_phase_noalloc_equals_phase_twice(kind):
    assert torch.cuda.is_available()
    if kind == "snp_llr":
        ws = [synth.snp_small(31, n_snp=4000, coverage=3.0), synth.snp_small(31, n_snp=1500, coverage=2.0)]
    else:
        ws = [synth.read_small(5, n_snp=400, n_reads=300, span=(10, 60)), synth.read_tiny()]
    for call, w in enumerate(ws):
        g = gpu_graph(w, kind, "f32")
        inf = g.info()
        if kind == "snp_llr":
            # several components, and the oracle agrees on their number
            assert inf["n_comp"] == oracle.components(oracle.build_graph(w, kind))[1] > 1
        s = _spins(inf["n"], 7 + call)
        h_ref, b_ref = qh.phase(g, s)
        # outputs pre-filled with garbage: every element must be written
        out = (torch.full((max(inf["n_snp"], 1),), 7, dtype=torch.int8, device="cuda"),
               torch.full((max(inf["n_snp"], 1),), 12345, dtype=torch.int32, device="cuda"))
        h, b = qh.phase(g, s, noalloc=True, out=out)
        torch.cuda.synchronize()
        assert torch.equal(h, h_ref), call
        assert torch.equal(b, b_ref), call
        if kind == "snp_llr":
            ho, bo = oracle.phase_parity(*oracle.components(oracle.build_graph(w, kind)), cpu(s), w.init_h1)
            assert np.array_equal(cpu(h), ho) and np.array_equal(cpu(b), bo)
        g.free()
