"""Per-species GP blocks (eq. 1: one GP per descriptor type; a descriptor per
central species gives one GP per species) through the C ABI: each species'
rows (FP64 and BF16X3) against the oracle, a two-species model fitted with
its blocks side by side (one-shot and through the fold calls) against the
oracle's fit of the concatenated system, and its prediction as the sum of the
species blocks' predictions."""
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
    h = gapx.Gap(0)
    yield h
    h.close()


def close(got, ref, tol, what):
    err = np.abs(np.asarray(got) - np.asarray(ref)).max()
    scale = max(np.abs(ref).max(), 1e-300)
    assert err <= tol * scale, f"{what}: max err {err:.3e} vs scale {scale:.3e}"


def problem(w, seed=41):
    b = synth.generate(w)
    spc = np.random.default_rng(seed).integers(0, 2, b.n_atoms).astype(np.int32)
    rng = np.random.default_rng(seed + 1)
    # each species' sparse points drawn from its own atoms (bit copies)
    Xs = []
    for z, Mz in ((0, w.M), (1, w.M // 2 + 3)):
        idx = rng.choice(np.flatnonzero(spc == z), Mz, replace=False)
        Xs.append(b.desc[idx].astype(np.float64))
    return b, spc, Xs


@pytest.mark.parametrize("wname,D", [("fit_small", None), ("ragged", 37)])
def test_species_rows(gapx, gap, wname, D):
    w = synth.WORKLOADS["fit_small"] if wname == "fit_small" else \
        synth.Workload("species_ragged", 43, n_cfg=9, atoms_lo=1, atoms_hi=13, D=D, nb=5, M=15)
    b, spc, Xs = problem(w)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    st = torch.tensor(spc, device="cuda")
    for z, X in enumerate(Xs):
        sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
        ref = oracle.build_knm_species(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta,
                                       w.delta, spc, z)
        print(f"species rows {wname} z={z}: {ref.shape}", flush=True)
        for prec, tol in (("fp64", TOL), ("bf16x3", 1e-4)):
            A = gap.build_knm_species(atoms, sp, st, z, precision=prec)
            got = A[:X.shape[0], :b.n_rows].T.cpu().numpy()
            close(got[:b.n_cfg], ref[:b.n_cfg], tol, f"{prec} energy rows z={z}")
            close(got[b.n_cfg:], ref[b.n_cfg:], tol, f"{prec} force rows z={z}")


def test_two_species_fit_and_predict(gapx, gap):
    w = synth.WORKLOADS["fit_small"]
    b, spc, Xs = problem(w)
    M0, M1 = Xs[0].shape[0], Xs[1].shape[0]
    M = M0 + M1
    K = np.hstack([oracle.build_knm_species(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X,
                                            w.zeta, w.delta, spc, z) for z, X in enumerate(Xs)])
    Kmm = np.zeros((M, M))
    Kmm[:M0, :M0] = oracle.build_kmm(Xs[0], w.zeta, w.delta)
    Kmm[M0:, M0:] = oracle.build_kmm(Xs[1], w.zeta, w.delta)
    c_true = np.random.default_rng(5).standard_normal(M)
    sig = synth.sigma_rows(w, b.counts)
    y = K @ c_true + synth.noise(w, b.cfg_ids, b.counts)
    c_ref = oracle.fit(K, Kmm, y, sig, w.jitter)

    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    st = torch.tensor(spc, device="cuda")
    sps = [gapx.Sparse.from_host(X, w.zeta, w.delta) for X in Xs]
    Kmm_d = gapx.colmajor(M, M, M)
    K0 = gap.build_kmm(sps[0])
    K1 = gap.build_kmm(sps[1])
    Kmm_d[:M0, :M0] = K0
    Kmm_d[M0:, M0:] = K1
    yd, sd = torch.tensor(y, device="cuda"), torch.tensor(sig, device="cuda")
    # streamed: both blocks built side by side into the fold block area
    T = gap.fold_buffer(M, b.n_rows)
    gap.fold_init(T, M, Kmm_d, w.jitter)
    gap.build_knm_species(atoms, sps[0], st, 0, out=T, row0=M + 1, col0=0)
    gap.build_knm_species(atoms, sps[1], st, 1, out=T, row0=M + 1, col0=M0)
    gap.fold_rows(T, M, b.n_rows, yd, sd)
    c_fold, _, _ = gap.fold_solve(T, M)
    close(c_fold.cpu().numpy(), c_ref, TOL, "c of the two-species model (fold)")
    # one shot: the same blocks in one design buffer
    A = gapx.colmajor(b.n_rows + M, M + 1)
    gap.build_knm_species(atoms, sps[0], st, 0, out=A, col0=0)
    gap.build_knm_species(atoms, sps[1], st, 1, out=A, col0=M0)
    spM = gapx.Sparse(torch.zeros(M, sps[0].X.shape[1], dtype=torch.float64, device="cuda"), w.D,
                      w.zeta, w.delta)
    c_one, _ = gap.fit(A, b.n_rows, Kmm_d, yd, sd, w.jitter, spM)
    close(c_one.cpu().numpy(), c_ref, TOL, "c of the two-species model (one shot)")
    # the model's prediction: the sum of its species blocks
    cs = (c_fold[:M0], c_fold[M0:])
    e = torch.zeros(b.n_atoms, dtype=torch.float64, device="cuda")
    ec = torch.zeros(b.n_cfg, dtype=torch.float64, device="cuda")
    F = torch.zeros(b.n_atoms, 3, dtype=torch.float64, device="cuda")
    for z in (0, 1):
        pr = gap.predict_species(atoms, sps[z], cs[z], st, z, forces=True)
        e += pr["e_atom"]
        ec += pr["e_cfg"]
        F += pr["forces"]
        ez, _, _, _ = oracle.predict_species(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, None, Xs[z],
                                             cs[z].cpu().numpy(), w.zeta, w.delta, spc, z)
        close(pr["e_atom"].cpu().numpy(), ez, TOL, f"local energies of species {z}")
    Kc = K @ c_fold.cpu().numpy()
    close(ec.cpu().numpy(), Kc[:b.n_cfg], TOL, "model energies")
    close(F.cpu().numpy().reshape(-1), Kc[b.n_cfg:], TOL, "model forces")
