"""Bit-exact check of the BF16X3 split (reading of the split-BF16 contraction),
through the C ABI: hi = bf16(fp32(x)) and lo = bf16(fp32(x) - hi), every
rounding to nearest even, with the reference formed here from the IEEE bit
patterns (round to nearest even of the upper 16 bits of an FP32 word).  Covers
the Jacobian split kernel (FP32 and FP64 input) and the sparse-point split
kernel with its transposed halves, rounding ties included, so that a truncating
split or a lo formed from the FP64 value instead of its FP32 rounding fails."""
import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gap():
    import paper_2310_03921_amd as g
    assert torch.cuda.is_available(), "GPU tests need a gfx950 device"
    h = g.Gap(0)
    yield h
    h.close()


def rne_bf16_bits(f32):
    u = np.ascontiguousarray(f32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    return ((u + 0x7FFF + ((u >> 16) & 1)) >> 16).astype(np.uint16)


def bf16_value(bits):
    return (bits.astype(np.uint32) << 16).view(np.float32)


def reference_split(x):
    f = np.asarray(x).astype(np.float32)           # FP64 -> FP32, nearest even
    hi = rne_bf16_bits(f)
    rest = f - bf16_value(hi)                        # exact in FP32
    lo = rne_bf16_bits(rest)
    return hi, lo


def inputs(rows, cols, ld, dtype, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((rows, ld)) * 10.0 ** rng.integers(-12, 12, (rows, 1))
    # FP32 words whose low 16 bits are exactly half way (ties to even), for
    # both parities of the kept bits, and x - hi ties in the second split
    base = rng.standard_normal(rows * ld).astype(np.float32).view(np.uint32)
    tie = ((base & 0xFFFF0000) | 0x8000).view(np.float32).reshape(rows, ld)
    x[::3] = tie[::3]
    tie2 = ((base & 0xFFFFFF00) | 0x80).view(np.float32).reshape(rows, ld)
    x[1::3] = tie2[1::3]
    if dtype == np.float64:
        # doubles half way between two FP32 neighbours
        f = x[2::3].astype(np.float32)
        up = np.nextafter(f, np.float32(np.inf))
        x[2::3] = (f.astype(np.float64) + up.astype(np.float64)) / 2
    x[:, cols:] = 0.0
    return x.astype(dtype)


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
@pytest.mark.parametrize("rows,cols,ld", [(37, 37, 40), (96, 252, 252), (5, 1000, 1000)])
def test_split_rows_bit_exact(gap, dtype, rows, cols, ld):
    x = inputs(rows, cols, ld, dtype, seed=rows + cols)
    hi, lo, _, _ = gap.split_bf16x3(torch.tensor(x, device="cuda"), cols)
    hi = hi.cpu().numpy().view(np.uint16)
    lo = lo.cpu().numpy().view(np.uint16)
    rh, rl = reference_split(x[:, :cols])
    assert np.array_equal(hi[:, :cols], rh)
    assert np.array_equal(lo[:, :cols], rl)
    assert not hi[:, cols:].any() and not lo[:, cols:].any()
    # the pair keeps ~16 significant bits of the FP32 value
    f = x[:, :cols].astype(np.float32).astype(np.float64)
    back = bf16_value(rh).astype(np.float64) + bf16_value(rl).astype(np.float64)
    assert np.all(np.abs(back - f) <= 2.0 ** -16 * np.abs(f))


def test_split_sparse_points_transposed(gap):
    M, D, ld = 45, 70, 72
    x = inputs(M, D, ld, np.float64, seed=9)
    hi, lo, ht, lt = gap.split_bf16x3(torch.tensor(x, device="cuda"), D, transposed=True)
    hi, lo = hi.cpu().numpy().view(np.uint16), lo.cpu().numpy().view(np.uint16)
    ht, lt = ht.cpu().numpy().view(np.uint16), lt.cpu().numpy().view(np.uint16)
    rh, rl = reference_split(x[:, :D])
    assert np.array_equal(hi[:, :D], rh) and np.array_equal(lo[:, :D], rl)
    assert not hi[:, D:].any() and not lo[:, D:].any()
    assert np.array_equal(ht[:, :M], rh.T) and np.array_equal(lt[:, :M], rl.T)
    assert not ht[:, M:].any() and not lt[:, M:].any()
