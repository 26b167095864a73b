"""FP64 refinement by batches of rows (gap_refine_rows, gap_refine_solve)
through the C ABI against the FP64 oracle, |gpu - oracle| <= 1e-10 * max|oracle|:

* one step from a seeded c with the oracle's exact factor R: the rows' share
  of A^T r, r . r, and the corrected c (which is the least-squares solution);
* the streamed BF16X3 fit (rows folded batch by batch) refined with three
  steps over the same batches: c within 1e-10 of the oracle's FP64 fit, as
  gap_fit's own refinement of the one-shot BF16X3 fit;
* host-side refusals.
"""
import ctypes

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


def relmax(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    return np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300)


def batch_rows(b, c0, c1):
    """Row indices of configurations [c0, c1) in the batch's row order."""
    a0, a1 = int(b.cfg_ptr[c0]), int(b.cfg_ptr[c1])
    return np.concatenate([np.arange(c0, c1), b.n_cfg + np.arange(3 * a0, 3 * a1)])


def problem(w):
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    Kmm = oracle.build_kmm(X, w.zeta, w.delta)
    y = K @ synth.hidden_coefficients(w) + synth.noise(w, b.cfg_ids, b.counts)
    sig = synth.sigma_rows(w, b.counts)
    return b, X, K, Kmm, y, sig


def ragged():
    return synth.Workload("ragged", 33, n_cfg=9, atoms_lo=1, atoms_hi=23, D=37, nb=3, M=23,
                          zeta=3, delta=1.7)


@pytest.mark.parametrize("wname", ["fit_small", "ragged"])
def test_one_step_exact_r(gapx, gap, wname):
    w = ragged() if wname == "ragged" else synth.WORKLOADS[wname]
    b, X, K, Kmm, y, sig = problem(w)
    A, bb = oracle.design_matrix(K, Kmm, y, sig, w.jitter)
    R = oracle.augmented_r(A, bb)[:w.M, :w.M]
    c0 = np.random.default_rng(17).standard_normal(w.M)
    g_ref, rr_ref = oracle.refine_rows(K, y, sig, c0)
    c_ref = oracle.refine_solve(R, Kmm, w.jitter, g_ref, c0)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    g = torch.zeros(w.M, dtype=torch.float64, device="cuda")
    rr = torch.zeros(1, dtype=torch.float64, device="cuda")
    cd = torch.tensor(c0, device="cuda")
    cuts = [0, 1, 1, b.n_cfg // 2, b.n_cfg]   # an empty batch and a one-configuration one
    for k0, k1 in zip(cuts[:-1], cuts[1:]):
        rows = batch_rows(b, k0, k1)
        gap.refine_rows(atoms.configs(k0, k1), sp, cd, torch.tensor(y[rows], device="cuda"),
                        torch.tensor(sig[rows], device="cuda"), g, rr)
    gap.sync()
    assert relmax(g.cpu().numpy(), g_ref) <= TOL
    assert abs(float(rr[0]) - rr_ref) <= TOL * rr_ref
    Rd = gapx.colmajor(w.M, w.M, w.M)
    Rd.copy_(torch.tensor(R.T.copy(), device="cuda"))
    gap.refine_solve(Rd, w.M, torch.tensor(Kmm.T.copy(), device="cuda"), w.jitter, g, cd)
    assert relmax(cd.cpu().numpy(), c_ref) <= TOL


@pytest.mark.parametrize("wname", ["fit_small", "ragged"])
def test_cached_weights_step(gapx, gap, wname):
    # S kept by the caller (gap_refine_weights) and passed to every pass
    # (gap_refine_rows_s): S against the oracle's kernel-gradient scale, and
    # the rows' share of A^T r and r . r as in the uncached step
    w = ragged() if wname == "ragged" else synth.WORKLOADS[wname]
    b, X, K, Kmm, y, sig = problem(w)
    c0 = np.random.default_rng(18).standard_normal(w.M)
    g_ref, rr_ref = oracle.refine_rows(K, y, sig, c0)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    Sd = gap.refine_weights(atoms, sp).cpu().numpy()
    S_ref = oracle.poly_kernel_grad_scale(b.desc.astype(np.float64) @ X.T, w.zeta, w.delta)
    assert relmax(Sd[:, :w.M], S_ref) <= TOL
    assert not Sd[:, w.M:].any()
    g = torch.zeros(w.M, dtype=torch.float64, device="cuda")
    rr = torch.zeros(1, dtype=torch.float64, device="cuda")
    cd = torch.tensor(c0, device="cuda")
    cuts = [0, 1, b.n_cfg // 3, b.n_cfg]
    for k0, k1 in zip(cuts[:-1], cuts[1:]):
        rows = batch_rows(b, k0, k1)
        ab = atoms.configs(k0, k1)
        Sb = gap.refine_weights(ab, sp)
        for _ in range(2):   # the same S serves every pass
            gb = torch.zeros(w.M, dtype=torch.float64, device="cuda")
            gap.refine_rows_s(ab, sp, Sb, cd, torch.tensor(y[rows], device="cuda"),
                              torch.tensor(sig[rows], device="cuda"), gb)
        g += gb
        gap.refine_rows_s(ab, sp, Sb, cd, torch.tensor(y[rows], device="cuda"),
                          torch.tensor(sig[rows], device="cuda"), torch.zeros_like(g), rr)
    gap.sync()
    assert relmax(g.cpu().numpy(), g_ref) <= TOL
    assert abs(float(rr[0]) - rr_ref) <= TOL * rr_ref


def test_streamed_mixed_fit_refined(gapx, gap):
    w = synth.WORKLOADS["fit_small_mixed"]
    b, X, K, Kmm, y, sig = problem(w)
    c_fit = oracle.fit(K, Kmm, y, sig, w.jitter)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    M = w.M
    Kmm_d = gap.build_kmm(sp)
    cuts = [0, 17, 33, b.n_cfg]
    batches = [(k0, k1, batch_rows(b, k0, k1)) for k0, k1 in zip(cuts[:-1], cuts[1:])]
    T = gap.fold_buffer(M, max(len(r) for _, _, r in batches))
    gap.fold_init(T, M, Kmm_d, w.jitter)
    dev = [(atoms.configs(k0, k1), torch.tensor(y[r], device="cuda"),
            torch.tensor(sig[r], device="cuda")) for k0, k1, r in batches]
    for (ab, yb, sb), (_, _, r) in zip(dev, batches):
        gap.build_knm_block(ab, sp, T, precision="bf16x3")
        gap.fold_rows(T, M, len(r), yb, sb)
    c, _, _ = gap.fold_solve(T, M)
    err0 = np.linalg.norm(c.cpu().numpy() - c_fit) / np.linalg.norm(c_fit)
    errs = []
    Ss = [gap.refine_weights(ab, sp) for ab, _, _ in dev]
    c2 = c.clone()
    for step in range(3):
        g = torch.zeros(M, dtype=torch.float64, device="cuda")
        for ab, yb, sb in dev:
            gap.refine_rows(ab, sp, c, yb, sb, g)
        gap.refine_solve(T, M, Kmm_d, w.jitter, g, c)
        errs.append(np.linalg.norm(c.cpu().numpy() - c_fit) / np.linalg.norm(c_fit))
        # the same steps with the batches' S kept between passes
        g2 = torch.zeros(M, dtype=torch.float64, device="cuda")
        for (ab, yb, sb), Sb in zip(dev, Ss):
            gap.refine_rows_s(ab, sp, Sb, c2, yb, sb, g2)
        gap.refine_solve(T, M, Kmm_d, w.jitter, g2, c2)
    assert np.linalg.norm((c2 - c).cpu().numpy()) <= TOL * np.linalg.norm(c_fit)
    print(f"\nstreamed BF16X3 fit: c rel {err0:.2e} -> " + " -> ".join(f"{e:.2e}" for e in errs))
    assert err0 > 1e-9 and errs[-1] <= TOL
    # gap_fit's own refinement of the one-shot BF16X3 fit reaches the same c
    A = gap.build_knm(atoms, sp, precision="bf16x3")
    c1, _ = gap.fit(A, b.n_rows, Kmm_d, torch.tensor(y, device="cuda"),
                    torch.tensor(sig, device="cuda"), w.jitter, sp, train=atoms, refine_steps=3)
    assert np.linalg.norm((c1 - c).cpu().numpy()) <= TOL * np.linalg.norm(c_fit)


def test_refine_host_checks(gapx, gap):
    L = gapx.lib()
    w = synth.WORKLOADS["fit_small"]
    b, X, K, Kmm, y, sig = problem(w)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, None)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    a, s = atoms.struct(), sp.struct()
    c = torch.zeros(w.M, dtype=torch.float64, device="cuda")
    g = torch.zeros(w.M, dtype=torch.float64, device="cuda")
    yd = torch.tensor(y, device="cuda")
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    bad = gapx.GAP_E_INVALID
    # no Jacobians, then no g
    assert L.gap_refine_rows(gap._h, ctypes.byref(a), ctypes.byref(s), p(c), p(yd), p(yd), p(g),
                             None) == bad
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    a = atoms.struct()
    assert L.gap_refine_rows(gap._h, ctypes.byref(a), ctypes.byref(s), p(c), p(yd), p(yd), None,
                             None) == bad
    Kd = torch.tensor(Kmm, device="cuda")
    R = gapx.colmajor(w.M, w.M, w.M)
    assert L.gap_refine_solve(gap._h, p(R), w.M - 1, w.M, p(Kd), 0.0, p(g), p(c)) == bad
    assert L.gap_refine_solve(gap._h, p(R), w.M, w.M, p(Kd), -1.0, p(g), p(c)) == bad
    # a zero R is refused after the solve, and the handle still works
    assert L.gap_refine_solve(gap._h, p(R), w.M, w.M, p(Kd), 0.0, p(g), p(c)) == gapx.GAP_E_RANK
    Kmm_d = gap.build_kmm(sp)
    assert relmax(Kmm_d.cpu().numpy().T, Kmm) <= TOL
