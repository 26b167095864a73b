"""Local-property rows (per-atom observations selected by a mask) through the
C ABI against the FP64 oracle: |gpu - oracle| <= 1e-10 * max|oracle|."""
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


def close(got, ref, tol, what):
    got, ref = np.asarray(got, np.float64), np.asarray(ref, np.float64)
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max()
    assert err <= tol * scale, f"{what}: rel err {err / scale:.3e}"


def ragged():
    return synth.Workload("ragged", 23, n_cfg=9, atoms_lo=1, atoms_hi=23, D=37, nb=3, M=23,
                          zeta=3, delta=1.7)


def masked_atoms(n_atoms, seed):
    # about half of the atoms carry a property (in atom order), one repeated
    rng = np.random.default_rng(seed)
    idx = np.flatnonzero(rng.random(n_atoms) < 0.5)
    if idx.size == 0:
        idx = np.array([0])
    return np.concatenate([idx, idx[:1]]).astype(np.int32)


@pytest.mark.parametrize("wname,ddt", [("fit_small", None), ("fit_small", "f32"),
                                       ("ragged", None)])
def test_local_rows_vs_oracle(gapx, gap, wname, ddt):
    w = ragged() if wname == "ragged" else synth.WORKLOADS[wname]
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    desc = b.desc.astype(np.float32) if ddt == "f32" else b.desc
    atoms = gapx.Atoms.from_host(b.cfg_ptr, desc, b.pair_ptr, b.pair_j, None,
                                 desc_dtype=torch.float32 if ddt == "f32" else None)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    idx = masked_atoms(b.n_atoms, 3)
    K = gap.build_local_rows(atoms, sp, torch.tensor(idx, device="cuda"))
    gap.sync()
    ref = oracle.build_local_rows(desc, X, idx, w.zeta, w.delta)
    close(K[:w.M, :len(idx)].T.cpu().numpy(), ref, TOL, "local rows")


def test_fit_with_local_rows_below_knm(gapx, gap):
    # energies, forces and a local property in one design buffer and one fit
    w = synth.WORKLOADS["fit_small"]
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    M = w.M
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    idx = masked_atoms(b.n_atoms, 7)
    KL = oracle.build_local_rows(b.desc, X, idx, w.zeta, w.delta)
    cstar = synth.hidden_coefficients(w)
    Kall = np.vstack([K, KL])
    rng = np.random.default_rng(4)
    y = Kall @ cstar + 1e-3 * rng.standard_normal(Kall.shape[0])
    sig = np.concatenate([synth.sigma_rows(w, b.counts), np.full(len(idx), 0.01)])
    Kmm = oracle.build_kmm(X, w.zeta, w.delta)
    c_ref = oracle.fit(Kall, Kmm, y, sig, w.jitter)

    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    n = Kall.shape[0]
    A = gapx.colmajor(n + M, M + 1)
    gap.build_knm(atoms, sp, out=A)
    gap.build_local_rows(atoms, sp, torch.tensor(idx, device="cuda"), out=A, row0=b.n_rows)
    c, _ = gap.fit(A, n, gap.build_kmm(sp), torch.tensor(y, device="cuda"),
                   torch.tensor(sig, device="cuda"), w.jitter, sp)
    close(c.cpu().numpy(), c_ref, TOL, "c")
    # the predicted local property of the masked atoms is e_atom
    pr = gap.predict(atoms, sp, c, e_atom=True, e_cfg=False, forces=False)
    close(pr["e_atom"].cpu().numpy()[idx], KL @ c_ref, TOL, "e_atom of masked atoms")


def test_local_rows_bad_index(gapx, gap):
    w = ragged()
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, None)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    idx = torch.tensor([0, b.n_atoms, 1], dtype=torch.int32, device="cuda")
    K = gap.build_local_rows(atoms, sp, idx)
    with pytest.raises(gapx.GapError) as e:
        gap.sync()
    assert e.value.status == gapx.GAP_E_INVALID
    Kh = K[:w.M, :3].T.cpu().numpy()
    assert np.all(Kh[1] == 0.0)
    close(Kh[[0, 2]], oracle.build_local_rows(b.desc, X, [0, 1], w.zeta, w.delta), TOL, "valid rows")
