"""Predictive variance of local energies through the C ABI against the FP64
oracle.  var_i is a difference of terms of size k(d_i, d_i), so the bound is
|gpu - oracle| <= 1e-10 * max_i k(d_i, d_i), the FP64 bar on those terms."""
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


@pytest.fixture(scope="module")
def gap(gapx):
    return gapx.Gap(0)


def problem(w):
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    Kmm = oracle.build_kmm(X, w.zeta, w.delta)
    sig = synth.sigma_rows(w, b.counts)
    y = K @ synth.hidden_coefficients(w) + synth.noise(w, b.cfg_ids, b.counts)
    return b, X, K, Kmm, y, sig


def check(var_gpu, b, X, K, Kmm, y, sig, w):
    A, bb = oracle.design_matrix(K, Kmm, y, sig, w.jitter)
    R = oracle.augmented_r(A, bb)[:w.M, :w.M]
    ref = oracle.predict_variance(b.desc, X, Kmm, w.jitter, R, w.zeta, w.delta)
    d = b.desc.astype(np.float64)
    kii = w.delta ** 2 * np.sum(d * d, axis=1) ** w.zeta
    err = np.abs(var_gpu - ref).max() / kii.max()
    assert err <= 1e-10, err


def test_variance_after_fit(gapx, gap):
    w = synth.WORKLOADS["fit_small"]
    b, X, K, Kmm, y, sig = problem(w)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    Kmm_d = gap.build_kmm(sp)
    A = gap.build_knm(atoms, sp)
    gap.fit(A, b.n_rows, Kmm_d, torch.tensor(y, device="cuda"), torch.tensor(sig, device="cuda"),
            w.jitter, sp)
    var = gap.predict_variance(atoms, sp, Kmm_d, w.jitter, A)
    check(var.cpu().numpy(), b, X, K, Kmm, y, sig, w)


def test_variance_from_fold_state_ragged(gapx, gap):
    w = synth.Workload("ragged", 31, n_cfg=9, atoms_lo=1, atoms_hi=23, D=37, nb=3, M=23,
                       zeta=3, delta=1.7)
    b, X, K, Kmm, y, sig = problem(w)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    Kmm_d = gap.build_kmm(sp)
    M, n = w.M, b.n_rows
    T = gap.fold_buffer(M, n)
    gap.fold_init(T, M, Kmm_d, w.jitter)
    gap.build_knm_block(atoms, sp, T)
    gap.fold_rows(T, M, n, torch.tensor(y, device="cuda"), torch.tensor(sig, device="cuda"))
    var = gap.predict_variance(atoms, sp, Kmm_d, w.jitter, T)
    check(var.cpu().numpy(), b, X, K, Kmm, y, sig, w)
