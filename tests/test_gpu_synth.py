"""The device input generator against its host definition: Philox4x32-10 words
bit-exact (across the 2^32 counter boundary), the FP32 Box-Muller normals
within FP32 transcendental error of the host FP64 transform, and a batch's
Jacobians equal, bit for bit, to each of its configurations drawn alone."""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def device():
    assert torch.cuda.is_available(), "GPU tests need a gfx950 device"
    torch.cuda.set_device(0)


@pytest.mark.parametrize("g0", [0, (1 << 32) - 1000])
def test_device_words_bit_exact(g0):
    n = 4096
    dev = synth.device_words(11, synth.JAC_TAG, g0, n).cpu().numpy().view(np.uint32)
    host = synth.stream_words(11, synth.JAC_TAG, g0, n)
    assert np.array_equal(dev, host)


@pytest.mark.parametrize("e0,rows,D,ld", [(0, 300, 1500, 1500), (8, 97, 37, 40), (5, 11, 6, 8)])
def test_device_normals(e0, rows, D, ld):
    out = torch.full((rows, ld), -7.0, dtype=torch.float32, device="cuda")
    synth.device_normal_rows(out, 5, synth.JAC_TAG, e0, D, 0.1)
    got = out.cpu().numpy()
    e = e0 + np.arange(rows * D)
    g_lo, g_hi = e[0] // 4, e[-1] // 4
    z = synth.box_muller(synth.stream_words(5, synth.JAC_TAG, int(g_lo), int(g_hi - g_lo + 1)))
    ref = 0.1 * z.ravel()[e - 4 * g_lo].reshape(rows, D)
    # FP32 log / sqrt / hardware sine and cosine against the FP64 transform
    assert np.abs(got[:, :D] - ref).max() <= 1e-5
    assert np.all(got[:, D:] == -7.0)


def test_jacobians_of_a_batch_equal_each_configuration_alone():
    w = synth.WORKLOADS["fit_large_mixed"].with_(D=40)
    J = synth.device_jacobians(w, 10, 16)
    gptr = synth.global_atom_offsets(w)
    base = int(gptr[10]) * w.nb
    for c in (10, 13, 15):
        one = synth.device_jacobians(w, c, c + 1)
        p0 = int(gptr[c]) * w.nb - base
        assert torch.equal(J[p0:p0 + one.shape[0]], one)
    v = J[:, :, :w.D].double()
    assert abs(float(v.mean())) < 2e-3 and abs(float(v.std()) - 0.1) < 2e-3
