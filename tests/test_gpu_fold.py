"""Streamed fit (row blocks folded into the triangular factor) through the C ABI
against the FP64 oracle.

Same bar as the one-shot fit: |gpu - oracle| <= 1e-10 * max|oracle| for c.
The factor itself is unique only up to the sign of each row, so it is checked
through what is sign-free: the Gram matrix T^T T of the augmented system
(backward-stable QR: 1e-11 relative), |diag T| and the residual corner.
"""
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


def problem(w):
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    Kmm = oracle.build_kmm(X, w.zeta, w.delta)
    sig = synth.sigma_rows(w, b.counts)
    y = K @ synth.hidden_coefficients(w) + synth.noise(w, b.cfg_ids, b.counts)
    return b, X, K, Kmm, y, sig


def state_host(T, M):
    return T[:M + 1, :M + 1].T.cpu().numpy()


def oracle_fold(K, Kmm, y, sig, jitter, blocks):
    T = oracle.fold_init(Kmm, jitter)
    for r0, r1 in blocks:
        T = oracle.fold_rows(T, K[r0:r1], y[r0:r1], sig[r0:r1])
    return T


def check_state(T_gpu, T_orc, K, Kmm, y, sig, jitter):
    M = Kmm.shape[0]
    A, b = oracle.design_matrix(K, Kmm, y, sig, jitter)
    Ab = np.column_stack([A, b])
    G = Ab.T @ Ab
    assert np.all(np.tril(T_gpu, -1) == 0.0)
    gram_err = np.linalg.norm(T_gpu.T @ T_gpu - G) / np.linalg.norm(G)
    assert gram_err <= 1e-11, gram_err
    close(np.abs(np.diag(T_gpu)), np.abs(np.diag(T_orc)), 1e-8, "|diag T|")
    assert abs(abs(T_gpu[M, M]) - abs(T_orc[M, M])) <= 1e-9 * abs(T_orc[M, M])


def fold_rows_from(gap, T, M, Kd, y, sig, r0, r1):
    """Copy rows [r0, r1) of a device K_NM (col-major (M, ld) tensor) into the block area, fold."""
    n = r1 - r0
    if n > 0:
        T[:M, M + 1:M + 1 + n] = Kd[:M, r0:r1]
    gap.fold_rows(T, M, n, torch.tensor(y[r0:r1], device="cuda"),
                  torch.tensor(sig[r0:r1], device="cuda"))


@pytest.mark.parametrize("wname,cuts", [
    ("fit_small", [0, 700, 701, 1500, None]),
    ("ragged", [0, 0, 1, 2, 50, None]),
])
def test_fold_row_blocks_vs_oracle(gapx, gap, wname, cuts):
    if wname == "ragged":
        w = synth.Workload("ragged", 21, n_cfg=9, atoms_lo=1, atoms_hi=23, D=37, nb=3, M=23,
                           zeta=3, delta=1.3)
    else:
        w = synth.WORKLOADS[wname]
    b, X, K, Kmm, y, sig = problem(w)
    n = b.n_rows
    cuts = [n if c is None else min(c, n) for c in cuts]
    blocks = [(cuts[i], cuts[i + 1]) for i in range(len(cuts) - 1)]
    M = w.M
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    Kd = gap.build_knm(atoms, sp)
    T = gap.fold_buffer(M, max(r1 - r0 for r0, r1 in blocks))
    gap.fold_init(T, M, gap.build_kmm(sp), w.jitter)
    for r0, r1 in blocks:
        fold_rows_from(gap, T, M, Kd, y, sig, r0, r1)
    c, res, rd = gap.fold_solve(T, M)
    c_ref = oracle.fit(K, Kmm, y, sig, w.jitter)
    close(c.cpu().numpy(), c_ref, TOL, "c")
    T_orc = oracle_fold(K, Kmm, y, sig, w.jitter, blocks)
    check_state(state_host(T, M), T_orc, K, Kmm, y, sig, w.jitter)
    _, res_ref = oracle.fold_solve(T_orc)
    assert abs(res - res_ref) <= 1e-9 * res_ref
    assert rd[0] > 0 and rd[1] >= rd[0]


def sub_batch(b, c0, c1):
    """Configurations [c0, c1) of a host batch as arrays for Atoms.from_host."""
    a0, a1 = int(b.cfg_ptr[c0]), int(b.cfg_ptr[c1])
    p0, p1 = int(b.pair_ptr[a0]), int(b.pair_ptr[a1])
    return (b.cfg_ptr[c0:c1 + 1] - a0, b.desc[a0:a1], b.pair_ptr[a0:a1 + 1] - p0,
            b.pair_j[p0:p1] - a0, b.jac[p0:p1]), (a0, a1)


def test_fold_config_groups_built_in_place(gapx, gap):
    # K_NM rows of each group of configurations built by gap_build_knm straight
    # into the block area; the rows of a group are its energies then its forces.
    w = synth.WORKLOADS["fit_small"]
    b, X, K, Kmm, y, sig = problem(w)
    M, nc = w.M, b.n_cfg
    groups = [(0, 17), (17, 18), (18, nc)]
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    rows_of = []
    for c0, c1 in groups:
        _, (a0, a1) = sub_batch(b, c0, c1)
        rows_of.append(np.concatenate([np.arange(c0, c1), nc + np.arange(3 * a0, 3 * a1)]))
    T = gap.fold_buffer(M, max(len(r) for r in rows_of))
    gap.fold_init(T, M, gap.build_kmm(sp), w.jitter)
    full = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    for i, ((c0, c1), rows) in enumerate(zip(groups, rows_of)):
        if i % 2 == 0:  # device views of the resident batch
            atoms = full.configs(c0, c1)
        else:           # a batch uploaded from host arrays of the group
            arrs, _ = sub_batch(b, c0, c1)
            atoms = gapx.Atoms.from_host(*arrs)
        assert atoms.n_rows == len(rows)
        gap.build_knm_block(atoms, sp, T)
        gap.fold_rows(T, M, len(rows), torch.tensor(y[rows], device="cuda"),
                      torch.tensor(sig[rows], device="cuda"))
    c, res, _ = gap.fold_solve(T, M)
    close(c.cpu().numpy(), oracle.fit(K, Kmm, y, sig, w.jitter), TOL, "c")
    perm = np.concatenate(rows_of)
    T_orc = oracle_fold(K[perm], Kmm, y[perm], sig[perm], w.jitter, [(0, len(perm))])
    check_state(state_host(T, M), T_orc, K, Kmm, y, sig, w.jitter)


def test_fold_single_block_equals_fit(gapx, gap):
    w = synth.WORKLOADS["fit_small"]
    b, X, K, Kmm, y, sig = problem(w)
    M, n = w.M, b.n_rows
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    Kmm_d = gap.build_kmm(sp)
    yd, sd = torch.tensor(y, device="cuda"), torch.tensor(sig, device="cuda")
    A = gap.build_knm(atoms, sp)
    c_fit, _ = gap.fit(A, n, Kmm_d, yd, sd, w.jitter, sp)
    T = gap.fold_buffer(M, n)
    gap.fold_init(T, M, Kmm_d, w.jitter)
    gap.build_knm_block(atoms, sp, T)
    gap.fold_rows(T, M, n, yd, sd)
    c, res, _ = gap.fold_solve(T, M)
    close(c.cpu().numpy(), c_fit.cpu().numpy(), TOL, "fold vs fit")
    A_h, b_h = oracle.design_matrix(K, Kmm, y, sig, w.jitter)
    c_ref = oracle.fit(K, Kmm, y, sig, w.jitter)
    r_ref = np.linalg.norm(b_h - A_h @ c_ref)
    assert abs(res - r_ref) <= 1e-9 * r_ref


def test_fold_argument_errors(gapx, gap):
    M = 8
    T = gap.fold_buffer(M, 4)
    Kmm = torch.eye(M, dtype=torch.float64, device="cuda")
    gap.fold_init(T, M, Kmm, 0.0)
    before = T.clone()
    gap.fold_rows(T, M, 0, torch.zeros(1, dtype=torch.float64, device="cuda"),
                  torch.ones(1, dtype=torch.float64, device="cuda"))
    torch.cuda.synchronize()
    assert torch.equal(T, before)  # an empty block changes nothing
    with pytest.raises(gapx.GapError) as e:  # block larger than the buffer: host check
        gap.fold_rows(T, M, T.shape[1] - M, torch.zeros(T.shape[1], dtype=torch.float64,
                                                        device="cuda"),
                      torch.ones(T.shape[1], dtype=torch.float64, device="cuda"))
    assert e.value.status == gapx.GAP_E_INVALID
    bad = -torch.eye(M, dtype=torch.float64, device="cuda")
    with pytest.raises(gapx.GapError) as e:
        gap.fold_init(T, M, bad, 0.0)
    assert e.value.status == gapx.GAP_E_NOT_PD
