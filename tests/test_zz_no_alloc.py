"""gap_forces_noalloc (no device allocation inside the library; scratch in a
static device array) against gap_forces, through the C ABI: two calls in a row,
the second on a smaller input, then an input beyond the scratch limit, which the
host must refuse before anything is enqueued."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gapx():
    import paper_2310_03921_amd as g
    assert torch.cuda.is_available(), "GPU tests need a gfx950 device"
    return g


def _case(gapx, w, jac_dtype, seed):
    b = synth.generate(w)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac,
                                 jac_dtype=jac_dtype)
    g = np.random.default_rng(seed).standard_normal((b.n_atoms, w.D))
    return b, atoms, g


def test_noalloc_matches_forces_twice(gapx):
    gap = gapx.Gap(0)
    big = synth.Workload("noalloc_big", 71, n_cfg=40, atoms_lo=8, atoms_hi=64, D=252, nb=20, M=8)
    small = synth.Workload("noalloc_small", 72, n_cfg=5, atoms_lo=1, atoms_hi=9, D=37, nb=3, M=8)
    for w, jdt, seed in ((big, torch.float64, 1), (small, torch.float32, 2)):
        b, atoms, g = _case(gapx, w, jdt, seed)
        print(f"noalloc case {w.name}: {b.n_atoms} atoms, {b.n_pairs} pairs, D={w.D}", flush=True)
        gd = torch.tensor(g, device="cuda")
        ref = gap.forces(atoms, gd)
        out = torch.full((b.n_atoms, 3), float("nan"), dtype=torch.float64, device="cuda")
        gap.forces_noalloc(atoms, gd, out)
        gap.sync()
        # same kernels, same order of summation: identical results
        assert torch.equal(out, ref)
        jac = b.jac.astype(np.float32).astype(np.float64) if jdt == torch.float32 else b.jac
        # the oracle's forces from the same descriptor gradients g
        src = oracle.pair_sources(b.pair_ptr)
        Fg = np.zeros((b.n_atoms, 3))
        np.add.at(Fg, np.asarray(b.pair_j, np.int64), -np.einsum("pad,pd->pa", jac, g[src]))
        assert np.abs(out.cpu().numpy() - Fg).max() <= 1e-10 * np.abs(Fg).max()
    gap.close()


def test_noalloc_refuses_beyond_scratch(gapx):
    gap = gapx.Gap(0)
    w = synth.Workload("noalloc_tiny", 73, n_cfg=2, atoms_lo=2, atoms_hi=3, D=8, nb=2, M=4)
    b, atoms, g = _case(gapx, w, torch.float64, 3)
    a = atoms.struct()
    a.n_pairs = 4_000_000   # 32 bytes a pair: beyond the 64 MiB scratch
    gd = torch.tensor(g, device="cuda")
    out = torch.zeros(b.n_atoms, 3, dtype=torch.float64, device="cuda")
    st = gapx.lib().gap_forces_noalloc(gap._h, ctypes.byref(a), ctypes.c_void_p(gd.data_ptr()),
                                       ctypes.c_void_p(out.data_ptr()))
    assert st == gapx.GAP_E_INVALID
    assert b"scratch" in gapx.lib().gap_last_error(gap._h)
    gap.sync()
    assert torch.all(out == 0)
    gap.close()
