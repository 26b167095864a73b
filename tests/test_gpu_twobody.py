"""Two-body squared-exponential descriptor through the C ABI against the FP64
oracle (|gpu - oracle| <= 1e-10 * max|oracle|), and a model of two descriptors
(dot-product SOAP-like block beside a two-body block, K_MM block-diagonal)
fitted through the fold calls."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

TOL = 1e-10
PAR = dict(delta=1.3, theta=0.6, r_cut=4.5, width=1.0)


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
    return synth.Workload("ragged", 41, n_cfg=9, atoms_lo=1, atoms_hi=23, D=37, nb=3, M=23,
                          zeta=3, delta=1.7)


def k2_of(gapx, x, par=PAR):
    return gapx.SE2b.from_host(x, delta=par["delta"], theta=par["theta"], r_cut=par["r_cut"],
                               cut_width=par["width"])


@pytest.mark.parametrize("wname,M2", [("fit_small", 24), ("ragged", 70)])
def test_2b_rows_kmm_predict_vs_oracle(gapx, gap, wname, M2):
    w = ragged() if wname == "ragged" else synth.WORKLOADS[wname]
    b = synth.generate(w, jac=False)
    r = synth.pair_vectors(w, b)
    x = synth.sparse_distances(w, M2)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, None)
    k2 = k2_of(gapx, x)
    rd = torch.tensor(r, device="cuda")
    K = gap.build_2b_rows(atoms, k2, rd)
    ref = oracle.build_2b_rows(b.cfg_ptr, b.pair_ptr, b.pair_j, r, x, **PAR)
    Kh = K[:M2, :b.n_rows].T.cpu().numpy()
    close(Kh[:b.n_cfg], ref[:b.n_cfg], TOL, "2b energy rows")
    close(Kh[b.n_cfg:], ref[b.n_cfg:], TOL, "2b force rows")
    Kmm = gap.build_kmm_2b(k2).cpu().numpy().T
    assert np.array_equal(Kmm, Kmm.T)
    close(Kmm, oracle.build_kmm_2b(x, **PAR), TOL, "2b K_MM")
    c = np.random.default_rng(2).standard_normal(M2)
    pr = gap.predict_2b(atoms, k2, rd, torch.tensor(c, device="cuda"))
    E, F = oracle.predict_2b(b.cfg_ptr, b.pair_ptr, b.pair_j, r, x, c, **PAR)
    close(pr["e_cfg"].cpu().numpy(), E, TOL, "2b energies")
    close(pr["forces"].cpu().numpy(), F, TOL, "2b forces")


def test_two_descriptor_fit_through_fold(gapx, gap):
    # columns [0, M1): dot-product kernel on the descriptors; [M1, M1 + M2):
    # two-body SE kernel on the pair distances; K_MM = diag(K_MM^dp, K_MM^2b)
    w = synth.WORKLOADS["fit_small"]
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    r = synth.pair_vectors(w, b)
    # sparse distances inside the cutoff and spaced beyond theta, so that the
    # two-body K_MM is well conditioned (cond ~ 3e3) and the fit's solution is
    # determined to the FP64 bar; the rows tests above cover distances past the cutoff
    M1, M2 = w.M, 8
    x = synth.sparse_distances(w, M2, 0.5, 4.0)
    K1 = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    par = dict(PAR, theta=0.3)
    K2 = oracle.build_2b_rows(b.cfg_ptr, b.pair_ptr, b.pair_j, r, x, **par)
    K = np.hstack([K1, K2])
    Kmm = np.zeros((M1 + M2, M1 + M2))
    Kmm[:M1, :M1] = oracle.build_kmm(X, w.zeta, w.delta)
    Kmm[M1:, M1:] = oracle.build_kmm_2b(x, **par)
    c_true = np.concatenate([synth.hidden_coefficients(w), 0.3 * np.ones(M2)])
    sig = synth.sigma_rows(w, b.counts)
    y = K @ c_true + synth.noise(w, b.cfg_ids, b.counts)
    c_ref = oracle.fit(K, Kmm, y, sig, w.jitter)

    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    k2 = k2_of(gapx, x, par)
    rd = torch.tensor(r, device="cuda")
    M = M1 + M2
    Kmm_d = gapx.colmajor(M, M, M)
    gap.build_kmm(sp, out=Kmm_d)              # top-left block (ld M)
    gap.build_kmm_2b(k2, out=Kmm_d, row0=M1, col0=M1)
    T = gap.fold_buffer(M, b.n_rows)
    gap.fold_init(T, M, Kmm_d, w.jitter)
    gap.build_knm_block(atoms, sp, T, M=M, col0=0)
    gap.build_2b_block(atoms, k2, rd, T, M=M, col0=M1)
    gap.fold_rows(T, M, b.n_rows, torch.tensor(y, device="cuda"), torch.tensor(sig, device="cuda"))
    c, res, _ = gap.fold_solve(T, M)
    close(c.cpu().numpy(), c_ref, TOL, "c of the two-descriptor model")
    # the model's prediction is the sum of its two parts
    p1 = gap.predict(atoms, sp, c[:M1], e_atom=False, e_cfg=True, forces=True)
    p2 = gap.predict_2b(atoms, k2, rd, c[M1:])
    close((p1["e_cfg"] + p2["e_cfg"]).cpu().numpy(), K[:b.n_cfg] @ c_ref, TOL, "energies")
    close((p1["forces"] + p2["forces"]).cpu().numpy().reshape(-1), K[b.n_cfg:] @ c_ref, TOL,
          "forces")
