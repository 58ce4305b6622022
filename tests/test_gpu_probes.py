"""GPU tests of the ceiling probes (include/fastcod_probe.h): the atomic probe adds exactly one per
in-range index; the stream and lookup probes run over real workloads and leave their sink alone."""
import numpy as np
import pytest
import torch

from paper_2302_09247_amd import synth

pytestmark = pytest.mark.gpu


def test_probe_atomics_counts_every_index(fc):
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    n_words = 1000
    idx = torch.randint(0, 1200, (200_003,), generator=g, device="cuda", dtype=torch.int32)
    target = torch.zeros(n_words, dtype=torch.int32, device="cuda")
    fc.probe_atomics(target, idx)
    torch.cuda.synchronize()
    ii = idx.cpu().numpy()
    exp = np.bincount(ii[ii < n_words], minlength=n_words)
    np.testing.assert_array_equal(target.cpu().numpy(), exp)


def test_probe_stream_and_lookup_run(fc):
    w = synth.make_07mm(S=200_000, device="cuda")
    vol = fc.Volume(w.roi, w.lab, w.N, w.M)
    fc.probe_stream(w.points)
    fc.probe_lookup(vol, w.points)
    fc.probe_lookup(vol, w.points, scale=synth.SR_SCALE)
    torch.cuda.synchronize()
    sr = synth.make_sr(S=20_000, device="cuda")
    fc.probe_lookup(vol, sr.points, scale=sr.scale)
    small = synth.make_tiny64(seed=2, S=1000, device="cuda")
    v2 = fc.Volume(small.roi, small.lab, small.N, small.M)
    fc.probe_lookup(v2, small.points)
    fc.probe_stream(small.points[:7])
    torch.cuda.synchronize()
    vol.close()
    v2.close()
