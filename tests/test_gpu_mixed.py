"""Split-BF16 (BF16x3) form against the FP64 oracle, and FP64 iterative refinement.

Bounds (relative to max|oracle| of each output block) follow from the split:
hi + lo keeps ~16 significant bits of each FP32-rounded operand, products
are accumulated in FP32 over D <= 256 terms, so K_NM, energies and gradients
carry relative errors of order 1e-5; the bounds below leave a factor ~10.
After refinement with an exact FP64 residual, c must match the FP64 solution
to the FP64 bound (1e-10).
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-4


@pytest.fixture(scope="module")
def gapx():
    import paper_2310_03921_amd as g
    assert torch.cuda.is_available(), "GPU tests need a gfx950 device"
    return g


@pytest.fixture(scope="module")
def gap(gapx):
    return gapx.Gap(0)


def relmax(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)


def setup(gapx, w):
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    return b, X, atoms, sp


@pytest.mark.parametrize("wname,jdt,limit", [("fit_small_mixed", "f64", 0),
                                             ("fit_small_mixed", "f32", 0),
                                             ("fit_small_mixed", "f32", 1), ("ragged", "f64", 0),
                                             ("wide", "f32", 0), ("wide", "f64", 0),
                                             ("wide", "f32", 1), ("wide", "f64", 1)])
def test_knm_bf16x3(gapx, gap, wname, jdt, limit):
    # limit = 1: a one-byte cap on the optional workspace, so the Jacobian rows
    # are split in registers instead of once up front (the other kernel path)
    gap.set_workspace_limit(limit)
    if wname == "ragged":
        w = synth.Workload("ragged", 31, n_cfg=9, atoms_lo=1, atoms_hi=23, D=37, nb=3, M=23,
                           zeta=3, delta=1.7, precision="bf16x3")
    elif wname == "wide":
        # descriptors longer than one LDS chunk (D % 4 == 0, a partial last
        # 32-block), a partial last 128-column tile, ragged atom counts
        w = synth.Workload("wide", 33, n_cfg=11, atoms_lo=1, atoms_hi=40, D=300 if jdt == "f32" else 260,
                           nb=7, M=150, precision="bf16x3", jac_dtype=jdt, desc_dtype=jdt)
    else:
        w = synth.WORKLOADS[wname].with_(jac_dtype=jdt, desc_dtype=jdt)
    b, X, atoms, sp = setup(gapx, w)
    A = gap.build_knm(atoms, sp, precision="bf16x3")
    got = A[:w.M, :b.n_rows].T.cpu().numpy()
    ref = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    e_e = relmax(got[:b.n_cfg], ref[:b.n_cfg])
    e_f = relmax(got[b.n_cfg:], ref[b.n_cfg:])
    print(f"\n{wname}/{jdt}/limit {limit}: K_E rel {e_e:.2e}, K_F rel {e_f:.2e}")
    gap.set_workspace_limit(0)
    assert e_e <= MIXED_TOL and e_f <= MIXED_TOL
    assert e_f > 0  # the split path really ran (not the FP64 kernels)


def test_fit_mixed_with_refinement(gapx, gap):
    """Precision form of the small fit: c, energy RMSE, force RMSE vs the FP64 oracle."""
    w = synth.WORKLOADS["fit_small_mixed"]
    b, X, atoms, sp = setup(gapx, w)
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    Kmm = oracle.build_kmm(X, w.zeta, w.delta)
    y = K @ synth.hidden_coefficients(w) + synth.noise(w, b.cfg_ids, b.counts)
    sig = synth.sigma_rows(w, b.counts)
    c_ref = oracle.fit(K, Kmm, y, sig, w.jitter)
    yd, sd = torch.tensor(y, device="cuda"), torch.tensor(sig, device="cuda")
    Kmm_d = gap.build_kmm(sp)
    out = {}
    for steps in (0, 3):
        A = gap.build_knm(atoms, sp, precision="bf16x3")
        c, info = gap.fit(A, b.n_rows, Kmm_d, yd, sd, w.jitter, sp, train=atoms,
                          refine_steps=steps)
        c = c.cpu().numpy()
        rel = np.linalg.norm(c - c_ref) / np.linalg.norm(c_ref)
        e_ref = K[:b.n_cfg] @ c_ref
        f_ref = K[b.n_cfg:] @ c_ref
        n_c = b.counts.astype(float)
        e_rmse = np.sqrt(np.mean(((K[:b.n_cfg] @ c - e_ref) / n_c) ** 2))
        f_rmse = np.sqrt(np.mean((K[b.n_cfg:] @ c - f_ref) ** 2))
        out[steps] = (rel, e_rmse, f_rmse, info["resid_norm"])
        print(f"\nrefine={steps}: c rel {rel:.2e}, energy RMSE {e_rmse:.2e}/atom, "
              f"force RMSE {f_rmse:.2e}, |A^T r| {info['resid_norm']}")
    assert out[0][0] <= 1e-4 and out[0][1] <= 1e-6 and out[0][2] <= 1e-5
    assert out[3][0] <= 1e-10
    rn = out[3][3]
    assert rn[-1] < rn[0]


def test_predict_bf16x3(gapx, gap):
    w = synth.WORKLOADS["fit_small"]
    b, X, atoms, sp = setup(gapx, w)
    c = np.random.default_rng(2).standard_normal(w.M)
    out = gap.predict(atoms, sp, torch.tensor(c, device="cuda"), precision="bf16x3", dEdd=True,
                      forces=True)
    e, ec, g, F = oracle.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, c, w.zeta,
                                 w.delta)
    for name, ref in (("e_atom", e), ("e_cfg", ec), ("dEdd", g), ("forces", F)):
        r = relmax(out[name].cpu().numpy(), ref)
        print(f"\npredict bf16x3 {name}: rel {r:.2e}")
        assert r <= MIXED_TOL, name


def test_backward_bf16x3(gapx, gap):
    w = synth.WORKLOADS["fit_small"]
    b, X, atoms, sp = setup(gapx, w)
    rng = np.random.default_rng(3)
    c = rng.standard_normal(w.M)
    ge = rng.standard_normal(b.n_atoms)
    dd, dc, dX = gap.predict_backward(atoms, sp, torch.tensor(c, device="cuda"),
                                      torch.tensor(ge, device="cuda"), precision="bf16x3")
    r_dd, r_dc, r_dX = oracle.predict_backward(b.desc, X, c, ge, w.zeta, w.delta)
    for name, got, ref in (("d_desc", dd, r_dd), ("d_c", dc, r_dc), ("d_X", dX, r_dX)):
        r = relmax(got.cpu().numpy(), ref)
        print(f"\nbackward bf16x3 {name}: rel {r:.2e}")
        assert r <= MIXED_TOL, name


@pytest.mark.parametrize("shape,ddt", [("ragged", "f64"), ("ragged", "f32"), ("tiles", "f32"),
                                       ("tiles", "f64")])
def test_predict_and_backward_bf16x3_ragged(gapx, gap, shape, ddt):
    # shapes that end inside every tile of the BF16X3 GEMM: D not a multiple
    # of 4 (a 4-entry group straddles D) nor of 32, M and N not multiples of
    # 32 or 256 (two row and two column tiles for "tiles"), FP32 and FP64
    # descriptors
    if shape == "ragged":
        w = synth.Workload("ragged_p", 41, n_cfg=9, atoms_lo=1, atoms_hi=23, D=37, nb=3, M=23,
                           zeta=3, delta=1.7, desc_dtype=ddt, jac_dtype=ddt)
    else:
        w = synth.Workload("tiles_p", 43, n_cfg=7, atoms_lo=40, atoms_hi=90, D=291, nb=4, M=301,
                           zeta=4, delta=0.9, desc_dtype=ddt, jac_dtype=ddt)
    b, X, atoms, sp = setup(gapx, w)
    rng = np.random.default_rng(5)
    c = rng.standard_normal(w.M)
    ge = rng.standard_normal(b.n_atoms)
    out = gap.predict(atoms, sp, torch.tensor(c, device="cuda"), precision="bf16x3", dEdd=True,
                      forces=True)
    e, ec, g, F = oracle.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, c, w.zeta,
                                 w.delta)
    dd, dc, dX = gap.predict_backward(atoms, sp, torch.tensor(c, device="cuda"),
                                      torch.tensor(ge, device="cuda"), precision="bf16x3")
    r_dd, r_dc, r_dX = oracle.predict_backward(b.desc, X, c, ge, w.zeta, w.delta)
    print(f"\n{shape} {ddt}: {b.n_atoms} atoms, D={w.D}, M={w.M}")
    for name, got, ref in (("e_atom", out["e_atom"], e), ("e_cfg", out["e_cfg"], ec),
                           ("dEdd", out["dEdd"], g), ("forces", out["forces"], F),
                           ("d_desc", dd, r_dd), ("d_c", dc, r_dc), ("d_X", dX, r_dX)):
        r = relmax(got.cpu().numpy(), ref)
        print(f"  {name}: rel {r:.2e}")
        assert r <= MIXED_TOL, name


def test_refinement_stops_once_converged(gapx, gap):
    # with room for seven steps, the refinement stops once the error it leaves
    # is predicted below 1e-14 (two or three steps for this system), and the
    # report holds one |A^T r| per step taken plus the final one
    w = synth.WORKLOADS["fit_small_mixed"]
    b, X, atoms, sp = setup(gapx, w)
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    Kmm = oracle.build_kmm(X, w.zeta, w.delta)
    y = K @ synth.hidden_coefficients(w) + synth.noise(w, b.cfg_ids, b.counts)
    sig = synth.sigma_rows(w, b.counts)
    c_ref = oracle.fit(K, Kmm, y, sig, w.jitter)
    A = gap.build_knm(atoms, sp, precision="bf16x3")
    c, info = gap.fit(A, b.n_rows, gap.build_kmm(sp), torch.tensor(y, device="cuda"),
                      torch.tensor(sig, device="cuda"), w.jitter, sp, train=atoms,
                      refine_steps=7)
    rel = np.linalg.norm(c.cpu().numpy() - c_ref) / np.linalg.norm(c_ref)
    print(f"\nrefinement stopped after {info['refine_done']} steps: c rel {rel:.2e}, "
          f"|A^T r| {info['resid_norm']}")
    assert 2 <= info["refine_done"] < 7
    assert len(info["resid_norm"]) == info["refine_done"] + 1
    assert rel <= 1e-10


def test_fit_without_the_final_residual(gapx, gap):
    # skipping the residual after the last step changes neither c nor the
    # steps taken; the report then holds the residuals before each step only
    w = synth.WORKLOADS["fit_small_mixed"]
    b, X, atoms, sp = setup(gapx, w)
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    y = torch.tensor(K @ synth.hidden_coefficients(w) + synth.noise(w, b.cfg_ids, b.counts),
                     device="cuda")
    sig = torch.tensor(synth.sigma_rows(w, b.counts), device="cuda")
    Kmm = gap.build_kmm(sp)
    out = {}
    try:
        for report in (True, False):
            gap.set_fit_report(report)
            A = gap.build_knm(atoms, sp, precision="bf16x3")
            out[report] = gap.fit(A, b.n_rows, Kmm, y, sig, w.jitter, sp, train=atoms,
                                  refine_steps=7)
    finally:
        gap.set_fit_report(True)
    (c1, i1), (c0, i0) = out[True], out[False]
    assert i0["refine_done"] == i1["refine_done"] >= 2
    assert torch.equal(c0, c1)
    assert len(i0["resid_norm"]) == i0["refine_done"]
    assert i0["resid_norm"] == i1["resid_norm"][:-1]
