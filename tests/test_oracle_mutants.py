"""Plant plausible mistakes in the oracle (CPU only) and check that a pin catches each.

A pin that no mutant can trip proves nothing; these keep the pins honest.
"""
import numpy as np
import pytest

import pins
from oracle import gap_oracle as G

_orig_knm = G.build_knm
_orig_grad = G.poly_kernel_grad_scale
_orig_kernel = G.poly_kernel
_orig_design = G.design_matrix
_orig_predict = G.predict
_orig_backward = G.predict_backward
_orig_pt = G.pair_transpose
_orig_fold_rows = G.fold_rows
_orig_augr = G.augmented_r
_orig_local = G.build_local_rows
_orig_virial = G.build_virial_rows
_orig_var = G.predict_variance
_orig_curlev = G.cur_leverage
_orig_dr = G.se2b_kernel_dr
_orig_2b = G.build_2b_rows
_orig_fcut = G.cutoff_fn
_orig_refine_rows = G.refine_rows
_orig_refine_solve = G.refine_solve
_orig_knm_species = G.build_knm_species
_orig_predict_species = G.predict_species


def knm_sign_flip(*a):
    K = _orig_knm(*a)
    n_cfg = len(a[0]) - 1
    K[n_cfg:] *= -1
    return K


def knm_drop_last_atom(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta):
    K = _orig_knm(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta)
    for c in range(len(cfg_ptr) - 1):
        if cfg_ptr[c + 1] - cfg_ptr[c] > 1:
            i = cfg_ptr[c + 1] - 1
            K[c] -= _orig_kernel(np.asarray(desc[i], float) @ np.asarray(X, float).T, zeta, delta)
    return K


def knm_scale_by_target(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta):
    # scale pairs by the kernel gradient of the target atom instead of the source
    swapped = G.pair_sources(pair_ptr)
    return _orig_knm(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta) if len(swapped) == 0 else \
        _scale_target(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta)


def _scale_target(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta):
    n_cfg = len(cfg_ptr) - 1
    K = _orig_knm(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta)
    X = np.asarray(X, float)
    P = np.asarray(desc, float) @ X.T
    S = _orig_grad(P, zeta, delta)
    src = G.pair_sources(pair_ptr)
    KF = np.zeros((int(cfg_ptr[-1]), 3, X.shape[0]))
    for p in range(len(pair_j)):
        KF[pair_j[p]] -= S[pair_j[p]][None, :] * (np.asarray(jac[p], float) @ X.T)
    K[n_cfg:] = KF.reshape(-1, X.shape[0])
    return K


def grad_wrong_power(p, zeta, delta):
    return delta * delta * zeta * np.asarray(p, float) ** zeta


def kernel_delta_not_squared(p, zeta, delta):
    return delta * np.asarray(p, float) ** zeta


def design_b_unscaled(Knm, Kmm, y, sigma, jitter):
    A, b = _orig_design(Knm, Kmm, y, sigma, jitter)
    b[:len(y)] = y
    return A, b


def design_no_jitter(Knm, Kmm, y, sigma, jitter):
    return _orig_design(Knm, Kmm, y, sigma, 0.0 if jitter > 0 else 1e-3)


def predict_forces_transposed(cfg_ptr, desc, pair_ptr, pair_j, jac, X, c, zeta, delta):
    e, ec, g, F = _orig_predict(cfg_ptr, desc, pair_ptr, pair_j, jac, X, c, zeta, delta)
    if F is not None:
        # accumulate on the source atom instead of the target atom
        src = G.pair_sources(pair_ptr)
        F2 = np.zeros_like(F)
        for p in range(len(src)):
            F2[src[p]] -= np.asarray(jac[p], float) @ g[src[p]]
        F = F2
    return e, ec, g, F


def backward_dx_missing_c(desc, X, c, g_e, zeta, delta):
    dD, dc, dX = _orig_backward(desc, X, c, g_e, zeta, delta)
    return dD, dc, dX / np.asarray(c, float)[:, None]


def pair_transpose_unstable(pair_ptr, pair_j, n_atoms):
    tptr, tpair = _orig_pt(pair_ptr, pair_j, n_atoms)
    for j in range(n_atoms):
        s = slice(tptr[j], tptr[j + 1])
        tpair[s] = tpair[s][::-1].copy()
    return tptr, tpair


def fold_rows_y_unscaled(T, Knm_block, y_block, sigma_block):
    return _orig_fold_rows(T, Knm_block, np.asarray(y_block, float) * np.asarray(sigma_block, float),
                           sigma_block)


def fold_rows_drops_state(T, Knm_block, y_block, sigma_block):
    # factor of the block alone: the rows folded before are lost
    return _orig_fold_rows(np.zeros_like(T), Knm_block, y_block, sigma_block)


def augmented_r_no_corner(A, b):
    T = _orig_augr(A, b)
    T[-1, -1] = 0.0
    return T


def local_rows_next_atom(desc, X, atom_idx, zeta, delta):
    n = np.asarray(desc).shape[0]
    return _orig_local(desc, X, (np.asarray(atom_idx) + 1) % n, zeta, delta)


def local_rows_gradient_scale(desc, X, atom_idx, zeta, delta):
    # the kernel-gradient scale in place of the kernel
    D = np.asarray(desc, float)[np.asarray(atom_idx, int)]
    return G.poly_kernel_grad_scale(D @ np.asarray(X, float).T, zeta, delta)


def virial_transposed(cfg_ptr, desc, pair_ptr, jac, pair_r, X, zeta, delta):
    K = _orig_virial(cfg_ptr, desc, pair_ptr, jac, pair_r, X, zeta, delta)
    n = K.shape[0] // 9
    return K.reshape(n, 3, 3, -1).transpose(0, 2, 1, 3).reshape(K.shape)


def virial_sign_flip(cfg_ptr, desc, pair_ptr, jac, pair_r, X, zeta, delta):
    return -_orig_virial(cfg_ptr, desc, pair_ptr, jac, pair_r, X, zeta, delta)


def variance_data_term_sign(desc, X, Kmm, jitter, R, zeta, delta):
    # subtract the data term instead of adding it
    base = _orig_var(desc, X, Kmm, jitter, np.eye(np.asarray(X).shape[0]) * 1e300, zeta, delta)
    full = _orig_var(desc, X, Kmm, jitter, R, zeta, delta)
    return base - (full - base)


def variance_prior_only(desc, X, Kmm, jitter, R, zeta, delta):
    # the prior variance k_ii, the sparse-set term left out
    d = np.asarray(desc, float)
    return delta ** 2 * np.sum(d * d, axis=1) ** zeta + 0.0 * _orig_var(desc, X, Kmm, jitter, R,
                                                                       zeta, delta)


def variance_data_term_only(desc, X, Kmm, jitter, R, zeta, delta):
    # subset-of-regressors form k_i^T (A^T A)^-1 k_i: the k_ii - k_i^T K_MM^-1 k_i
    # part left out (inside [0, k_ii], so the bound alone does not catch it)
    d = np.asarray(desc, float)
    kii = delta ** 2 * np.sum(d * d, axis=1) ** zeta
    full = _orig_var(desc, X, Kmm, jitter, R, zeta, delta)
    base = _orig_var(desc, X, Kmm, jitter, np.eye(np.asarray(X).shape[0]) * 1e300, zeta, delta)
    return full - base + 0.0 * kii


def cur_leverage_no_inverse(desc, jitter):
    d = np.asarray(desc, float)
    return np.sum(d * d, axis=1) / max(1.0, float(np.sum(d * d)) / d.shape[1])


def cur_leverage_inverse_squared(desc, jitter):
    # d^T G^-2 d in place of d^T G^-1 d
    Dm = np.asarray(desc, float)
    G = Dm.T @ Dm + jitter * np.eye(Dm.shape[1])
    Z = np.linalg.solve(G, Dm.T).T
    return np.sum(Z * Z, axis=1)


def se2b_dr_no_cutoff_slope(r, x, delta, theta, r_cut, width):
    # drops the f_cut'(r) term of dk/dr
    rr = np.asarray(r, dtype=np.float64)
    e = delta ** 2 * G.cutoff_fn(x, r_cut, width) * np.exp(-(rr - x) ** 2 / (2.0 * theta ** 2))
    return -e * G.cutoff_fn(rr, r_cut, width) * (rr - x) / theta ** 2


def build_2b_rows_target_sign(cfg_ptr, pair_ptr, pair_j, pair_r, x, delta, theta, r_cut, width):
    K = _orig_2b(cfg_ptr, pair_ptr, pair_j, pair_r, x, delta, theta, r_cut, width)
    n_cfg = len(cfg_ptr) - 1
    src = G.pair_sources(pair_ptr)
    R = np.asarray(pair_r, float)
    for p in range(len(src)):
        r = float(np.linalg.norm(R[p]))
        if r > 0:
            dk = _orig_dr(r, x, delta, theta, r_cut, width)
            j = int(pair_j[p])
            for a in range(3):
                K[n_cfg + 3 * j + a] += dk * R[p, a] / r   # target term added instead of subtracted
    return K


def cutoff_half_width(r, r_cut, width):
    return _orig_fcut(r, r_cut, 0.5 * width)


def refine_rows_unweighted(Knm_rows, y, sigma, c):
    # A^T r without the second Sigma^-1/2
    K = np.asarray(Knm_rows, float)
    w = 1.0 / np.asarray(sigma, float)
    r = w * (np.asarray(y, float) - K @ c)
    return K.T @ r, float(r @ r)


def refine_solve_no_jitter(R, Kmm, jitter, g, c):
    return _orig_refine_solve(R, Kmm, 0.0, g, c)


def refine_solve_regulariser_sign(R, Kmm, jitter, g, c):
    c = np.asarray(c, float)
    return _orig_refine_solve(R, -np.asarray(Kmm, float), -jitter, g, c)


def species_mask_by_target(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta, species, z):
    # force rows kept for pairs whose TARGET has species z (energy rows right)
    K = _orig_knm_species(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta, species, z)
    Kall = _orig_knm(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta)
    n_cfg = len(cfg_ptr) - 1
    tmask = np.repeat((np.asarray(species) == z).astype(float), 3)[:, None]
    K[n_cfg:] = tmask * Kall[n_cfg:]
    return K


def species_forces_unmasked(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta, species, z):
    # energy rows masked, force rows of every centre
    K = _orig_knm_species(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta, species, z)
    Kall = _orig_knm(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta)
    n_cfg = len(cfg_ptr) - 1
    K[n_cfg:] = Kall[n_cfg:]
    return K


def predict_species_unmasked_gradient(cfg_ptr, desc, pair_ptr, pair_j, jac, X, c, zeta, delta,
                                      species, z):
    # local energies masked, descriptor gradients (and so forces) of every atom
    e, ec, _, _ = _orig_predict_species(cfg_ptr, desc, pair_ptr, pair_j, jac, X, c, zeta, delta,
                                        species, z)
    _, _, g, F = _orig_predict(cfg_ptr, desc, pair_ptr, pair_j, jac, X, c, zeta, delta)
    return e, ec, g, F


MUTANTS = [
    ("build_knm", knm_sign_flip),
    ("build_knm_species", species_mask_by_target),
    ("build_knm_species", species_forces_unmasked),
    ("predict_species", predict_species_unmasked_gradient),
    ("build_knm", knm_drop_last_atom),
    ("build_knm", knm_scale_by_target),
    ("poly_kernel_grad_scale", grad_wrong_power),
    ("poly_kernel", kernel_delta_not_squared),
    ("design_matrix", design_b_unscaled),
    ("design_matrix", design_no_jitter),
    ("predict", predict_forces_transposed),
    ("predict_backward", backward_dx_missing_c),
    ("pair_transpose", pair_transpose_unstable),
    ("fold_rows", fold_rows_y_unscaled),
    ("fold_rows", fold_rows_drops_state),
    ("augmented_r", augmented_r_no_corner),
    ("build_local_rows", local_rows_next_atom),
    ("build_local_rows", local_rows_gradient_scale),
    ("build_virial_rows", virial_transposed),
    ("build_virial_rows", virial_sign_flip),
    ("predict_variance", variance_data_term_sign),
    ("predict_variance", variance_prior_only),
    ("predict_variance", variance_data_term_only),
    ("cur_leverage", cur_leverage_no_inverse),
    ("cur_leverage", cur_leverage_inverse_squared),
    ("se2b_kernel_dr", se2b_dr_no_cutoff_slope),
    ("build_2b_rows", build_2b_rows_target_sign),
    ("cutoff_fn", cutoff_half_width),
    ("refine_rows", refine_rows_unweighted),
    ("refine_solve", refine_solve_no_jitter),
    ("refine_solve", refine_solve_regulariser_sign),
]


@pytest.mark.parametrize("name,mutant", MUTANTS, ids=[m[1].__name__ for m in MUTANTS])
def test_some_pin_catches_mutant(monkeypatch, name, mutant):
    monkeypatch.setattr(G, name, mutant)
    caught = []
    for check in pins.ALL_CHECKS:
        try:
            check(G)
        except (AssertionError, np.linalg.LinAlgError, ValueError, RuntimeError):
            caught.append(check.__name__)
    assert caught, f"no pin catches mutant {mutant.__name__}"
