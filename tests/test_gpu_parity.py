"""HIP path (through the C ABI) against the FP64 oracle, element by element.

Tolerance of the FP64 path: |gpu - oracle| <= 1e-10 * max|oracle| per output
block (energy rows, force rows, c, energies, forces, gradients), the relative
bound the method's FP64 form is held to; integer outputs bit-exact.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-10


@pytest.fixture(scope="module")
def gapx():
    import paper_2310_03921_amd as g
    assert torch.cuda.is_available(), "GPU tests need a gfx950 device"
    return g


@pytest.fixture(scope="module")
def gap(gapx):
    return gapx.Gap(0)


def close(got, ref, tol=TOL, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    scale = max(np.abs(ref).max(), 1e-300) if ref.size else 1.0
    err = np.abs(got - ref).max() if ref.size else 0.0
    assert err <= tol * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e} (rel {err / scale:.3e})"


def knm_host(A, n_rows, M):
    return A[:M, :n_rows].T.cpu().numpy()


def batch_and_sparse(w):
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    return b, X


def to_device(gapx, b, X, w, jac_dtype=None, desc_dtype=None):
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac,
                                 desc_dtype=desc_dtype, jac_dtype=jac_dtype)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    return atoms, sp


# --------------------------------------------------------------- hand example
def test_hand_example(gapx, gap):
    with open(os.path.join(HERE, "golden", "hand_example.json")) as f:
        g = json.load(f)
    atoms = gapx.Atoms.from_host(np.array(g["cfg_ptr"]), np.array(g["desc"]),
                                 np.array(g["pair_ptr"]), np.array(g["pair_j"], np.int32),
                                 np.array(g["jac"]))
    sp = gapx.Sparse.from_host(np.array(g["X"]), g["zeta"], g["delta"])
    Kmm = gap.build_kmm(sp).cpu().numpy().T
    close(Kmm, g["Kmm"], 1e-14, "Kmm")
    A = gap.build_knm(atoms, sp)
    close(knm_host(A, atoms.n_rows, sp.M), g["Knm"], 1e-14, "Knm")
    out = gap.predict(atoms, sp, torch.tensor(g["c"], dtype=torch.float64, device="cuda"),
                      dEdd=True, forces=True)
    close(out["e_atom"].cpu(), g["e_atom"], 1e-14, "e_atom")
    close(out["e_cfg"].cpu(), g["e_cfg"], 1e-14, "e_cfg")
    close(out["dEdd"].cpu(), g["dEdd"], 1e-14, "dEdd")
    close(out["forces"].cpu(), g["forces"], 1e-14, "forces")


# ------------------------------------------------------------ pair transpose
@pytest.mark.parametrize("wname", ["fit_small"])
def test_pair_transpose_bit_exact(gapx, gap, wname):
    w = synth.WORKLOADS[wname]
    b, X = batch_and_sparse(w)
    atoms, _ = to_device(gapx, b, X, w)
    tptr, tpair = gap.pair_transpose(atoms)
    rptr, rpair = oracle.pair_transpose(b.pair_ptr, b.pair_j, b.n_atoms)
    assert np.array_equal(tptr.cpu().numpy(), rptr)
    assert np.array_equal(tpair.cpu().numpy(), rpair)


def test_pair_transpose_empty(gapx, gap):
    atoms = gapx.Atoms.from_host(np.array([0, 3]), np.eye(3, 4), np.zeros(4, np.int64),
                                 np.zeros(0, np.int32), None)
    tptr, tpair = gap.pair_transpose(atoms)
    assert np.array_equal(tptr.cpu().numpy(), np.zeros(4, np.int64))
    assert tpair.numel() == 0


# ----------------------------------------------------------------- K_MM, K_NM
def test_kmm_exact_symmetry_and_parity(gapx, gap):
    w = synth.WORKLOADS["fit_small"]
    X = synth.sparse_points(w)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    K = gap.build_kmm(sp).cpu().numpy().T
    assert np.array_equal(K, K.T)
    close(K, oracle.build_kmm(X, w.zeta, w.delta), TOL, "Kmm")
    assert np.linalg.eigvalsh(K).min() > 0


@pytest.mark.parametrize("jdt", [None, "f32"])
def test_knm_fit_small(gapx, gap, jdt):
    w = synth.WORKLOADS["fit_small"]
    if jdt == "f32":
        w = w.with_(jac_dtype="f32", desc_dtype="f32")
    b, X = batch_and_sparse(w)
    atoms, sp = to_device(gapx, b, X, w)
    A = gap.build_knm(atoms, sp)
    got = knm_host(A, b.n_rows, w.M)
    ref = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    close(got[:b.n_cfg], ref[:b.n_cfg], TOL, "energy rows")
    close(got[b.n_cfg:], ref[b.n_cfg:], TOL, "force rows")


def ragged_workload(seed=21):
    # D and M off the tile sizes, 1-atom configurations, atoms with no pairs
    return synth.Workload("ragged", seed, n_cfg=9, atoms_lo=1, atoms_hi=23, D=37, nb=3, M=23,
                          zeta=3, delta=1.7)


def test_knm_ragged_edges(gapx, gap):
    w = ragged_workload()
    b, X = batch_and_sparse(w)
    # give atom 0 no pairs and make one pair point at its own source
    keep = np.ones(b.n_pairs, bool)
    keep[:w.nb] = False
    pair_ptr = np.concatenate([[0], np.cumsum(np.diff(b.pair_ptr) - np.bincount(
        np.repeat(np.arange(b.n_atoms), np.diff(b.pair_ptr))[~keep], minlength=b.n_atoms))])
    pair_j = b.pair_j[keep].copy()
    jac = b.jac[keep]
    pair_j[0] = 1  # source atom 1 -> itself
    ref = oracle.build_knm(b.cfg_ptr, b.desc, pair_ptr, pair_j, jac, X, w.zeta, w.delta)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, pair_ptr, pair_j, jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    got = knm_host(gap.build_knm(atoms, sp), b.n_rows, w.M)
    close(got, ref, TOL, "ragged K_NM")


def test_knm_no_pairs_at_all(gapx, gap):
    w = ragged_workload(22)
    b, X = batch_and_sparse(w)
    pair_ptr = np.zeros(b.n_atoms + 1, np.int64)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, pair_ptr, np.zeros(0, np.int32), None)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    got = knm_host(gap.build_knm(atoms, sp), b.n_rows, w.M)
    ref = oracle.build_knm(b.cfg_ptr, b.desc, pair_ptr, np.zeros(0, np.int32),
                           np.zeros((0, 3, w.D)), X, w.zeta, w.delta)
    close(got, ref, TOL, "no-pair K_NM")
    assert np.all(got[b.n_cfg:] == 0)


def test_knm_permutation(gapx, gap):
    import pins
    w = synth.WORKLOADS["fit_small"].with_(n_cfg=12)
    b, X = batch_and_sparse(w)
    atoms, sp = to_device(gapx, b, X, w)
    K1 = knm_host(gap.build_knm(atoms, sp), b.n_rows, w.M)
    desc, pptr, pj, jac, perm = pins.permuted_batch(b, np.random.default_rng(3))
    atoms2 = gapx.Atoms.from_host(b.cfg_ptr, desc, pptr, pj, jac)
    K2 = knm_host(gap.build_knm(atoms2, sp), b.n_rows, w.M)
    close(K2[:b.n_cfg], K1[:b.n_cfg], 1e-13, "energy rows under permutation")
    rows = b.n_cfg + 3 * np.repeat(perm, 3) + np.tile(np.arange(3), b.n_atoms)
    close(K2[rows], K1[b.n_cfg:], 1e-13, "force rows under permutation")


def test_knm_deterministic(gapx, gap):
    w = synth.WORKLOADS["fit_small"]
    b, X = batch_and_sparse(w)
    atoms, sp = to_device(gapx, b, X, w)
    K1 = knm_host(gap.build_knm(atoms, sp), b.n_rows, w.M)
    K2 = knm_host(gap.build_knm(atoms, sp), b.n_rows, w.M)
    assert np.array_equal(K1, K2)


# ------------------------------------------------------------------ fit / QR
def fit_problem(w):
    b, X = batch_and_sparse(w)
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    Kmm = oracle.build_kmm(X, w.zeta, w.delta)
    cstar = synth.hidden_coefficients(w)
    sig = synth.sigma_rows(w, b.counts)
    y = K @ cstar + synth.noise(w, b.cfg_ids, b.counts)
    return b, X, K, Kmm, y, sig


def test_fit_small_fp64(gapx, gap):
    w = synth.WORKLOADS["fit_small"]
    b, X, K, Kmm, y, sig = fit_problem(w)
    c_ref = oracle.fit(K, Kmm, y, sig, w.jitter)
    atoms, sp = to_device(gapx, b, X, w)
    Kmm_d = gap.build_kmm(sp)
    A = gap.build_knm(atoms, sp)
    c, info = gap.fit(A, b.n_rows, Kmm_d, torch.tensor(y, device="cuda"),
                      torch.tensor(sig, device="cuda"), w.jitter, sp)
    close(c.cpu().numpy(), c_ref, TOL, "c")
    assert info["min_abs_rdiag"] > 0


def test_fit_refinement_keeps_fp64_solution(gapx, gap):
    w = synth.WORKLOADS["fit_small"]
    b, X, K, Kmm, y, sig = fit_problem(w)
    c_ref = oracle.fit(K, Kmm, y, sig, w.jitter)
    atoms, sp = to_device(gapx, b, X, w)
    A = gap.build_knm(atoms, sp)
    c, info = gap.fit(A, b.n_rows, gap.build_kmm(sp), torch.tensor(y, device="cuda"),
                      torch.tensor(sig, device="cuda"), w.jitter, sp, train=atoms, refine_steps=2)
    close(c.cpu().numpy(), c_ref, TOL, "refined c")
    assert info["refine_done"] == 2 and len(info["resid_norm"]) == 3


def test_fit_not_pd_reported(gapx, gap):
    w = synth.WORKLOADS["fit_small"].with_(n_cfg=12)
    b, X = batch_and_sparse(w)
    atoms, sp = to_device(gapx, b, X, w)
    A = gap.build_knm(atoms, sp)
    bad = -torch.eye(w.M, dtype=torch.float64, device="cuda")
    with pytest.raises(gapx.GapError) as e:
        gap.fit(A, b.n_rows, bad, torch.ones(b.n_rows, dtype=torch.float64, device="cuda"),
                torch.ones(b.n_rows, dtype=torch.float64, device="cuda"), 0.0, sp)
    assert e.value.status == gapx.GAP_E_NOT_PD


# (600, 320) and (3000, 700) have several 128-wide outer blocks and a partial
# last one
@pytest.mark.parametrize("m,n,cond", [(300, 70, 1e2), (1000, 129, 1e2), (777, 200, 1e10),
                                      (64, 64, 1e3), (5000, 17, 10.0), (1500, 333, 1e6),
                                      (2100, 450, 1e3), (600, 320, 1e3), (3000, 700, 1e8)])
def test_lstsq_vs_lapack(gapx, gap, m, n, cond):
    rng = np.random.default_rng(m + n)
    U, _ = np.linalg.qr(rng.standard_normal((m, n)))
    V, _ = np.linalg.qr(rng.standard_normal((n, n)))
    s = np.logspace(0, -np.log10(cond), n)
    A = (U * s) @ V.T
    b = rng.standard_normal(m)
    ref = np.linalg.lstsq(A, b, rcond=None)[0]
    buf = gapx.colmajor(m, n + 1)
    buf[:n, :m] = torch.tensor(A.T)
    buf[n, :m] = torch.tensor(b)
    x, rd = gap.lstsq(buf, m, n)
    err = np.linalg.norm(x.cpu().numpy() - ref) / np.linalg.norm(ref)
    assert err <= max(TOL, cond * 1e-15 * 10), err


# ------------------------------------------------------- predict / backward
def test_predict_and_forces(gapx, gap):
    w = synth.WORKLOADS["fit_small"]
    b, X = batch_and_sparse(w)
    c = np.random.default_rng(5).standard_normal(w.M)
    atoms, sp = to_device(gapx, b, X, w)
    out = gap.predict(atoms, sp, torch.tensor(c, device="cuda"), dEdd=True, forces=True)
    e, ec, g, F = oracle.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, c, w.zeta, w.delta)
    close(out["e_atom"].cpu(), e, TOL, "e_atom")
    close(out["e_cfg"].cpu(), ec, TOL, "e_cfg")
    close(out["dEdd"].cpu(), g, TOL, "dEdd")
    close(out["forces"].cpu(), F, TOL, "forces")
    F2 = gap.forces(atoms, out["dEdd"])
    close(F2.cpu(), F, TOL, "gap_forces")


@pytest.mark.parametrize("D,jdt", [(300, None), (300, "f32"), (1024, "f32")])
def test_predict_forces_wide_descriptors(gapx, gap, D, jdt):
    # descriptor widths that take two and four 256-element segments per row in
    # the force contraction
    w = synth.Workload("wide", 17, n_cfg=5, atoms_lo=6, atoms_hi=19, D=D, nb=5, M=40)
    b, X = batch_and_sparse(w)
    jac = b.jac.astype(np.float32) if jdt == "f32" else b.jac
    c = synth.hidden_coefficients(w)
    e, ec, g, F = oracle.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, jac, X, c, w.zeta,
                                 w.delta)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, jac,
                                 jac_dtype=torch.float32 if jdt == "f32" else None)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    out = gap.predict(atoms, sp, torch.tensor(c, device="cuda"), e_atom=True, e_cfg=True,
                      dEdd=True, forces=True)
    close(out["e_atom"].cpu().numpy(), e, TOL, "e_atom")
    close(out["dEdd"].cpu().numpy(), g, TOL, "dEdd")
    close(out["forces"].cpu().numpy(), F, TOL, "forces")


def test_predict_ragged(gapx, gap):
    w = ragged_workload(23)
    b, X = batch_and_sparse(w)
    c = np.random.default_rng(6).standard_normal(w.M)
    atoms, sp = to_device(gapx, b, X, w)
    out = gap.predict(atoms, sp, torch.tensor(c, device="cuda"), dEdd=True, forces=True)
    e, ec, g, F = oracle.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, c, w.zeta, w.delta)
    close(out["e_atom"].cpu(), e, TOL, "e_atom")
    close(out["e_cfg"].cpu(), ec, TOL, "e_cfg")
    close(out["dEdd"].cpu(), g, TOL, "dEdd")
    close(out["forces"].cpu(), F, TOL, "forces")


@pytest.mark.parametrize("wname", ["fit_small", "ragged"])
def test_backward(gapx, gap, wname):
    w = synth.WORKLOADS[wname] if wname in synth.WORKLOADS else ragged_workload(24)
    b, X = batch_and_sparse(w)
    rng = np.random.default_rng(7)
    c = rng.standard_normal(w.M)
    ge = rng.standard_normal(b.n_atoms)
    atoms, sp = to_device(gapx, b, X, w)
    dd, dc, dX = gap.predict_backward(atoms, sp, torch.tensor(c, device="cuda"),
                                      torch.tensor(ge, device="cuda"))
    r_dd, r_dc, r_dX = oracle.predict_backward(b.desc, X, c, ge, w.zeta, w.delta)
    close(dd.cpu(), r_dd, TOL, "d_desc")
    close(dc.cpu(), r_dc, TOL, "d_c")
    close(dX.cpu(), r_dX, TOL, "d_X")


def test_autograd_function(gapx):
    w = ragged_workload(25)
    b, X = batch_and_sparse(w)
    rng = np.random.default_rng(8)
    c = rng.standard_normal(w.M)
    ge = rng.standard_normal(b.n_atoms)
    desc_t = torch.tensor(b.desc, device="cuda", requires_grad=True)
    X_t = torch.tensor(X, device="cuda", requires_grad=True)
    c_t = torch.tensor(c, device="cuda", requires_grad=True)
    e = gapx.gap_energy(desc_t, X_t, c_t, w.zeta, w.delta)
    e_ref, _, _, _ = oracle.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, None, X, c, w.zeta, w.delta)
    close(e.detach().cpu(), e_ref, TOL, "energies")
    (e * torch.tensor(ge, device="cuda")).sum().backward()
    r_dd, r_dc, r_dX = oracle.predict_backward(b.desc, X, c, ge, w.zeta, w.delta)
    close(desc_t.grad.cpu(), r_dd, TOL, "grad desc")
    close(c_t.grad.cpu(), r_dc, TOL, "grad c")
    close(X_t.grad.cpu(), r_dX, TOL, "grad X")
    # central finite differences in FP64 on a few entries
    h = 1e-6
    for (arr, grad, i, j) in ((desc_t, desc_t.grad, 1, 2), (X_t, X_t.grad, 3, 4)):
        with torch.no_grad():
            arr[i, j] += h
            ep = (gapx.gap_energy(desc_t, X_t, c_t, w.zeta, w.delta) * torch.tensor(ge, device="cuda")).sum()
            arr[i, j] -= 2 * h
            em = (gapx.gap_energy(desc_t, X_t, c_t, w.zeta, w.delta) * torch.tensor(ge, device="cuda")).sum()
            arr[i, j] += h
        fd = float((ep - em) / (2 * h))
        assert abs(fd - float(grad[i, j])) <= 1e-6 * max(1.0, abs(fd))
