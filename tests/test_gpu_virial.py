"""Virial rows through the C ABI against the FP64 oracle:
|gpu - oracle| <= 1e-10 * max|oracle|."""
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
    # D and M off the tile sizes, 1-atom configurations, atoms with no pairs
    return synth.Workload("ragged", 29, n_cfg=9, atoms_lo=1, atoms_hi=23, D=37, nb=3, M=23,
                          zeta=3, delta=1.7)


@pytest.mark.parametrize("wname,jdt", [("fit_small", None), ("fit_small", "f32"),
                                       ("ragged", None)])
def test_virial_rows_vs_oracle(gapx, gap, wname, jdt):
    w = ragged() if wname == "ragged" else synth.WORKLOADS[wname]
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    r = synth.pair_vectors(w, b)
    jac = b.jac.astype(np.float32) if jdt == "f32" else b.jac
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, jac,
                                 jac_dtype=torch.float32 if jdt == "f32" else None)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    Kv = gap.build_virial_rows(atoms, sp, torch.tensor(r, device="cuda"))
    gap.sync()
    ref = oracle.build_virial_rows(b.cfg_ptr, b.desc, b.pair_ptr, jac, r, X, w.zeta, w.delta)
    close(Kv[:w.M, :9 * b.n_cfg].T.cpu().numpy(), ref, TOL, "virial rows")


def test_fit_with_virial_rows(gapx, gap):
    # energies, forces and virials of every configuration in one design buffer
    w = synth.WORKLOADS["fit_small"]
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    r = synth.pair_vectors(w, b)
    M = w.M
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    KV = oracle.build_virial_rows(b.cfg_ptr, b.desc, b.pair_ptr, b.jac, r, X, w.zeta, w.delta)
    Kall = np.vstack([K, KV])
    rng = np.random.default_rng(6)
    y = Kall @ synth.hidden_coefficients(w) + 1e-3 * rng.standard_normal(Kall.shape[0])
    sig = np.concatenate([synth.sigma_rows(w, b.counts), np.full(KV.shape[0], 0.05)])
    c_ref = oracle.fit(Kall, oracle.build_kmm(X, w.zeta, w.delta), y, sig, w.jitter)

    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    n = Kall.shape[0]
    A = gapx.colmajor(n + M, M + 1)
    gap.build_knm(atoms, sp, out=A)
    gap.build_virial_rows(atoms, sp, torch.tensor(r, device="cuda"), out=A, row0=b.n_rows)
    c, _ = gap.fit(A, n, gap.build_kmm(sp), torch.tensor(y, device="cuda"),
                   torch.tensor(sig, device="cuda"), w.jitter, sp)
    close(c.cpu().numpy(), c_ref, TOL, "c")
