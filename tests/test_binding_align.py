"""Host-side checks of the binding's alignment handling (no GPU): the C ABI
refuses descriptor and Jacobian pointers that are not 32-byte aligned, so row
ranges that start 16 bytes off (FP32 rows of 252 or 1500 values at an odd row)
must reach it as aligned copies, and aligned ones as views."""
import numpy as np
import torch

import paper_2310_03921_amd as gapx


def test_aligned_view_copies_only_misaligned_rows():
    x = torch.zeros(10, 252, dtype=torch.float32)  # rows of 1008 bytes
    assert gapx._aligned(x)
    odd, even = x[1:], x[2:]
    assert not gapx._aligned(odd)                  # 1008 = 16 mod 32
    assert gapx._aligned(even)                     # 2016 = 0 mod 32
    v = gapx._aligned_view(odd)
    assert gapx._aligned(v) and v.data_ptr() != odd.data_ptr() and torch.equal(v, odd)
    assert gapx._aligned_view(even).data_ptr() == even.data_ptr()


def test_padded_rows_of_a_misaligned_slice():
    x = torch.arange(11 * 1500, dtype=torch.float32).reshape(11, 1500)
    y = gapx.padded_rows(x[1:], 1500)
    assert gapx._aligned(y) and torch.equal(y, x[1:])
    z = gapx.padded_rows(x[1:, :1499], 1499)       # padded to 1500 with zeros
    assert gapx._aligned(z) and z.shape == (10, 1500) and torch.all(z[:, 1499] == 0)


def test_configs_at_an_odd_atom_offset():
    rng = np.random.default_rng(5)
    counts = [3, 4, 2, 5]
    cfg_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    n, D, nb = int(cfg_ptr[-1]), 252, 2
    desc = torch.tensor(rng.standard_normal((n, D)), dtype=torch.float32)
    pair_ptr = torch.arange(0, nb * (n + 1), nb, dtype=torch.int64)
    pair_j = torch.tensor(np.concatenate([rng.integers(cfg_ptr[c], cfg_ptr[c + 1], nb * k)
                                          for c, k in enumerate(counts)]), dtype=torch.int32)
    jac = torch.tensor(rng.standard_normal((nb * n, 3, D)), dtype=torch.float32)
    at = gapx.Atoms(torch.tensor(cfg_ptr), desc, pair_ptr, pair_j, jac, D)
    sub = at.configs(1, 3)                          # atoms 3..8: an odd first row
    assert gapx._aligned(sub.desc) and gapx._aligned(sub.jac)
    assert torch.equal(sub.desc, desc[3:9]) and torch.equal(sub.jac, jac[6:18])
    assert sub.cfg_ptr.tolist() == [0, 4, 6]
    assert sub.pair_ptr[0] == 0 and int(sub.pair_j.min()) >= 0 and int(sub.pair_j.max()) < 6
    whole = at.configs(2, 4)                        # atoms 7..13
    assert gapx._aligned(whole.desc)
