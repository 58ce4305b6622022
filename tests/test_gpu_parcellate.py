"""GPU parity of the parcellation outputs (fastcod_parcellate) with the oracle, bit-exact: labels
and row sums are integers, and both sides take each fraction as the double quotient of two
integers rounded to float, so every output element must be equal."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from paper_2302_09247_amd import synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "parcellation_rows.json")


def _check(fc, C_np):
    C = torch.from_numpy(np.ascontiguousarray(C_np, np.int32)).cuda()
    lab, frac, sums = fc.parcellate(C)
    torch.cuda.synchronize()
    el, ef, es = oracle.parcellate(C_np.astype(np.int64))
    np.testing.assert_array_equal(lab.cpu().numpy(), el)
    np.testing.assert_array_equal(sums.cpu().numpy(), es)
    np.testing.assert_array_equal(frac.cpu().numpy().view(np.uint32), ef.view(np.uint32))


def test_golden_rows(fc):
    g = json.load(open(GOLDEN))
    C = np.array(g["C"])
    _check(fc, C)
    lab, _, _ = fc.parcellate(torch.from_numpy(C.astype(np.int32)).cuda())
    np.testing.assert_array_equal(lab.cpu().numpy(), g["labels"])


@pytest.mark.parametrize("shape,hi", [((1, 1), 5), ((7, 64), 3), ((100, 65), 1000), ((333, 180), 1 << 24),
                                      ((50, 360), (1 << 31) // 400), ((4000, 7), 2), ((3, 1000), 1 << 20),
                                      ((5, 128), 9), ((9, 256), 50), ((6, 257), 50), ((10, 129), 4),
                                      # more rows than the grid has wavefronts: each takes several,
                                      # the next one's entries loaded while the current is reduced
                                      ((20000, 37), 100), ((9000, 400), 1000)])
def test_random(fc, shape, hi):
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    C = rng.integers(0, hi, size=shape).astype(np.int64)
    C[rng.random(shape) < 0.5] = 0
    C[0] = 0
    if shape[1] > 3:
        C[-1, 1] = C[-1, 2] = C[-1].max() + 1   # a tie between two columns
    _check(fc, C)


def test_counted_matrix_and_null_outputs(fc):
    w = synth.make_125mm(S=200_000, device="cuda")
    C = fc.count(w.points, w.offsets, w.roi, w.lab, w.N, w.M)
    torch.cuda.synchronize()
    _check(fc, C.cpu().numpy().astype(np.int64))
    lab, frac, sums = fc.parcellate(C, fractions=False, sums=False)
    torch.cuda.synchronize()
    assert frac is None and sums is None
    np.testing.assert_array_equal(lab.cpu().numpy(), oracle.parcellate(C.cpu().numpy())[0])


def test_empty(fc):
    lab, frac, sums = fc.parcellate(torch.zeros((0, 4), dtype=torch.int32, device="cuda"))
    torch.cuda.synchronize()
    assert lab.numel() == 0 and frac.numel() == 0
