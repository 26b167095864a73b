"""The counter-based input generator (CPU side): Philox4x32-10 against the
known-answer vectors published with the generator (Salmon et al., SC'11,
Random123 kat_vectors), the Box-Muller transform's moments, and the device
library's exports (no GPU call)."""
import ctypes
import os

import numpy as np
import pytest

import synth

KAT = [
    ((0, 0, 0, 0), (0, 0), (0x6627E8D5, 0xE169C58D, 0xBC57AC4C, 0x9B00DBD8)),
    ((0xFFFFFFFF,) * 4, (0xFFFFFFFF,) * 2, (0x408F276D, 0x41C83B0E, 0xA20BC7C6, 0x6D5451FD)),
    ((0x243F6A88, 0x85A308D3, 0x13198A2E, 0x03707344), (0xA4093822, 0x299F31D0),
     (0xD16CFE09, 0x94FDCCEB, 0x5001E420, 0x24126EA1)),
]


@pytest.mark.parametrize("ctr,key,want", KAT)
def test_philox_known_answers(ctr, key, want):
    got = synth.philox4x32_10(np.array([ctr], dtype=np.uint32), *key)[0]
    assert tuple(int(x) for x in got) == want


def test_stream_counter_layout():
    # group g is counter (g mod 2^32, g / 2^32, 0, 0): the words of a range are
    # those of its groups computed one by one, across the 2^32 boundary too
    g0 = (1 << 32) - 2
    w = synth.stream_words(7, synth.JAC_TAG, g0, 4)
    for i in range(4):
        g = g0 + i
        one = synth.philox4x32_10(np.array([[g & 0xFFFFFFFF, g >> 32, 0, 0]], np.uint32), 7,
                                  synth.JAC_TAG)[0]
        assert np.array_equal(w[i], one)


def test_box_muller_moments():
    z = synth.box_muller(synth.stream_words(3, synth.JAC_TAG, 0, 250_000)).ravel()
    n = z.size
    assert abs(z.mean()) < 5 / np.sqrt(n)
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(np.mean(z ** 4) - 3.0) < 0.05


def test_device_library_exports():
    if not os.path.exists(synth._LIBSYNTH):
        pytest.skip("libsynth.so not built")
    L = ctypes.CDLL(synth._LIBSYNTH)
    assert hasattr(L, "synth_philox_words") and hasattr(L, "synth_normal_rows_f32")
