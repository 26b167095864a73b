"""CUR sparse-point selection through the C ABI against the FP64 oracle.

Leverage scores: |gpu - oracle| <= 1e-10 * max|oracle|.  The selection is an
index set decided by floating-point keys: it must equal the oracle's wherever
the keys leave no doubt (the n-th and (n+1)-th keys of the oracle further
apart than the leverage tolerance); otherwise every GPU pick must carry a key
no smaller than any key left out, within that tolerance."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def gapx():
    import paper_2310_03921_amd as g
    assert torch.cuda.is_available(), "GPU tests need a gfx950 device"
    return g


@pytest.fixture(scope="module")
def gap(gapx):
    return gapx.Gap(0)


def keys_of(lev, u):
    if u is None:
        return lev
    with np.errstate(divide="ignore"):
        return np.where(lev > 0, np.log(u) / lev, -np.inf)


def check_selection(got, ref_idx, key, n, tol):
    got = np.asarray(got, dtype=np.int64)
    assert len(got) == n and len(set(got.tolist())) == n
    order = np.lexsort((np.arange(len(key)), -key))
    if n < len(key) and key[order[n - 1]] - key[order[n]] > tol:
        assert set(got.tolist()) == set(ref_idx.tolist())
    left = np.setdiff1d(np.arange(len(key)), got)
    if len(left):
        assert key[got].min() >= key[left].max() - tol


@pytest.mark.parametrize("wname,ddt,jitter,use_u", [
    ("fit_small", None, 0.0, False),
    ("fit_small", "f32", 1e-8, True),
    ("ragged", None, 1e-6, False),
])
def test_cur_vs_oracle(gapx, gap, wname, ddt, jitter, use_u):
    w = (synth.Workload("ragged", 37, n_cfg=9, atoms_lo=1, atoms_hi=23, D=37, nb=3, M=23)
         if wname == "ragged" else synth.WORKLOADS[wname])
    b = synth.generate(w)
    desc = b.desc.astype(np.float32) if ddt == "f32" else b.desc
    atoms = gapx.Atoms.from_host(b.cfg_ptr, desc, b.pair_ptr, b.pair_j, None,
                                 desc_dtype=torch.float32 if ddt == "f32" else None)
    n = min(w.M, b.n_atoms)
    u = np.random.default_rng(3).random(b.n_atoms) if use_u else None
    idx, lev = gap.select_cur(atoms, n, jitter, None if u is None else torch.tensor(u, device="cuda"))
    ref_idx, ref_lev = oracle.cur_select(desc, n, jitter, u)
    lev = lev.cpu().numpy()
    err = np.abs(lev - ref_lev).max() / ref_lev.max()
    assert err <= TOL, err
    key = keys_of(ref_lev, u)
    check_selection(idx.cpu().numpy(), ref_idx, key, n, TOL * np.abs(key[np.isfinite(key)]).max())


def test_cur_unique_direction_first(gapx, gap):
    # an atom along a direction no other atom has: leverage 1, picked first
    rng = np.random.default_rng(5)
    Dm = rng.standard_normal((300, 8))
    Dm[:, 7] = 0.0
    Dm[123] = 0.0
    Dm[123, 7] = 3.0
    cfg_ptr = np.array([0, 300])
    pair_ptr = np.zeros(301, dtype=np.int64)
    atoms = gapx.Atoms.from_host(cfg_ptr, Dm, pair_ptr, np.zeros(0, dtype=np.int32), None)
    idx, lev = gap.select_cur(atoms, 10, 0.0)
    assert int(idx[0]) == 123
    assert abs(float(lev[123]) - 1.0) <= 1e-12
    assert abs(float(lev.sum()) - 8.0) <= 1e-10
