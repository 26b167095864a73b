"""The matrix-core throughput probe behind the measured peaks of the benchmark
line: every kind runs and reports a rate, random operands included, and a bad
kind is refused."""
import ctypes
import os

import pytest
import torch

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def probe():
    path = os.path.join(ROOT, "paper_2310_03921_amd", "libgap_peak.so")
    if not os.path.exists(path):
        pytest.fail("the probe library is not built")
    L = ctypes.CDLL(path)
    L.gap_peak_mfma.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)]
    L.gap_peak_mfma.restype = ctypes.c_int
    torch.cuda.set_device(0)
    return L


@pytest.mark.parametrize("kind,flop", [(0, 2048.0), (1, 16384.0), (2, 16384.0), (3, 2048.0)])
def test_every_kind_runs(probe, kind, flop):
    blocks, iters = 64, 1024
    out = torch.zeros(blocks * 256, dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ms, fl = ctypes.c_double(), ctypes.c_double()
    assert probe.gap_peak_mfma(st, kind, iters, blocks, ctypes.c_void_p(out.data_ptr()),
                               ctypes.byref(ms), ctypes.byref(fl)) == 0
    assert ms.value > 0
    assert fl.value == blocks * 4 * iters * 8 * flop
    assert bool(torch.isfinite(out).all())


def test_bad_arguments_refused(probe):
    out = torch.zeros(256, dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ms, fl = ctypes.c_double(), ctypes.c_double()
    for kind, iters in ((4, 16), (-1, 16), (0, 15), (0, 8)):
        assert probe.gap_peak_mfma(st, kind, iters, 1, ctypes.c_void_p(out.data_ptr()),
                                   ctypes.byref(ms), ctypes.byref(fl)) == -1
