"""Checks that pin the FP64 oracle to facts fixed by the paper and by mathematics.

Each check takes the oracle module (or a planted mutant of it) and raises
AssertionError when the fact does not hold.  They are independent of the
oracle's own arithmetic: complex-step and central finite differences of the
energy of a linearised descriptor, Euler's theorem for homogeneous functions,
ζ=1 / ζ=2 special cases computed through linearity and Kronecker products,
brute-force loops on tiny inputs, the normal-equation closed form (eq. GP_L),
an SVD least-squares solver, the full-GPR push-through identity, and the
delta / sigma scaling law.
"""
from __future__ import annotations

import numpy as np

import synth

TINY = synth.Workload("tiny", seed=11, n_cfg=4, atoms_lo=1, atoms_hi=5, D=6, nb=3, M=5,
                      zeta=4, delta=1.3)


def tiny_batch(w=TINY, seed=None):
    if seed is not None:
        w = w.with_(seed=seed)
    b = synth.generate(w, threads=1)
    X = synth.sparse_points(w, b)
    return w, b, X


def linearised_energy(w, b, X, cfg, m, dr):
    """E_c^m(r0 + dr) = delta^2 sum_{i in c} ((d_i + sum_k J_ik . dr_{j(i,k)}) . x_m)^zeta.

    dr is a complex array [N_at, 3]; the descriptor is linear in positions
    with slope given by the Jacobian slots (eq. for d eps / d r in Sec. Theory).
    Plain loops: independent of the oracle's GEMM/incidence structure.
    """
    a0, a1 = int(b.cfg_ptr[cfg]), int(b.cfg_ptr[cfg + 1])
    E = 0j
    for i in range(a0, a1):
        d = b.desc[i].astype(np.complex128)
        for p in range(int(b.pair_ptr[i]), int(b.pair_ptr[i + 1])):
            j = int(b.pair_j[p])
            for a in range(3):
                d = d + b.jac[p, a].astype(np.float64) * dr[j, a]
        s = 0j
        for k in range(w.D):
            s += d[k] * X[m, k]
        E += s ** w.zeta
    return w.delta ** 2 * E


def species_of(b, n_species=2, seed=31):
    """A seeded species label per atom (a stand-in for the element of a
    multi-species model)."""
    return np.random.default_rng(seed).integers(0, n_species, b.n_atoms).astype(np.int32)


def linearised_energy_species(w, b, X, cfg, m, dr, species, z):
    """linearised_energy with only the atoms of species z as centres (eq. 1:
    the local energies of one descriptor type's atoms).  Plain loops."""
    a0, a1 = int(b.cfg_ptr[cfg]), int(b.cfg_ptr[cfg + 1])
    E = 0j
    for i in range(a0, a1):
        if species[i] != z:
            continue
        d = b.desc[i].astype(np.complex128)
        for p in range(int(b.pair_ptr[i]), int(b.pair_ptr[i + 1])):
            j = int(b.pair_j[p])
            for a in range(3):
                d = d + b.jac[p, a].astype(np.float64) * dr[j, a]
        s = 0j
        for k in range(w.D):
            s += d[k] * X[m, k]
        E += s ** w.zeta
    return w.delta ** 2 * E


def check_kmm(orc):
    w, b, X = tiny_batch()
    K = orc.build_kmm(X, w.zeta, w.delta)
    assert np.array_equal(K, K.T), "K_MM not exactly symmetric"
    assert np.linalg.eigvalsh(K).min() > 0, "K_MM not positive definite"
    # unit-norm descriptors: k(x, x) = delta^2 (normalised kernel)
    assert np.allclose(np.diag(K), w.delta ** 2, rtol=1e-13, atol=0)
    # brute force entries
    for a in range(w.M):
        for c in range(w.M):
            s = sum(X[a, k] * X[c, k] for k in range(w.D))
            assert abs(K[a, c] - w.delta ** 2 * s ** w.zeta) <= 1e-14 * abs(w.delta ** 2)


def check_energy_rows_zeta1(orc):
    w, b, X = tiny_batch()
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, 1, w.delta)
    # zeta = 1: the energy row is linear, (sum_i d_i) . x_m
    for c in range(b.n_cfg):
        s = b.desc[b.cfg_ptr[c]:b.cfg_ptr[c + 1]].sum(axis=0)
        assert np.allclose(K[c], w.delta ** 2 * (X @ s), rtol=1e-13, atol=1e-15)


def check_energy_rows_zeta2(orc):
    w, b, X = tiny_batch()
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, 2, w.delta)
    # zeta = 2: (d . x)^2 = (d (x) d) . (x (x) x)
    for c in range(b.n_cfg):
        s = sum(np.kron(d, d) for d in b.desc[b.cfg_ptr[c]:b.cfg_ptr[c + 1]])
        ref = np.array([np.dot(s, np.kron(x, x)) for x in X]) * w.delta ** 2
        assert np.allclose(K[c], ref, rtol=1e-12, atol=1e-15)


def check_energy_rows_bruteforce(orc):
    w, b, X = tiny_batch()
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    zero = np.zeros((b.n_atoms, 3), dtype=np.complex128)
    for c in range(b.n_cfg):
        for m in range(w.M):
            ref = linearised_energy(w, b, X, c, m, zero).real
            assert abs(K[c, m] - ref) <= 1e-13 * max(1.0, abs(ref))


def check_sparse_self_entry(orc):
    w, b, X = tiny_batch()
    idx = synth.sparse_indices(w)
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    # a one-atom configuration made of a sparse atom has energy row entry delta^2 there
    one = np.array([0, 1], dtype=np.int64)
    for m, i in enumerate(idx):
        d = b.desc[i:i + 1]
        K1 = orc.build_knm(one, d, np.array([0, 0]), np.zeros(0, np.int32),
                           np.zeros((0, 3, w.D)), X, w.zeta, w.delta)
        assert abs(K1[0, m] - w.delta ** 2) <= 1e-13
        assert K1.shape == (4, w.M) and np.all(K1[1:] == 0)
    assert K.shape == (b.n_rows, w.M)


def check_force_rows_complex_step(orc, h=1e-30):
    w, b, X = tiny_batch()
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    for c in range(b.n_cfg):
        for j in range(int(b.cfg_ptr[c]), int(b.cfg_ptr[c + 1])):
            for a in range(3):
                dr = np.zeros((b.n_atoms, 3), dtype=np.complex128)
                dr[j, a] = 1j * h
                for m in range(w.M):
                    ref = -linearised_energy(w, b, X, c, m, dr).imag / h
                    got = K[b.n_cfg + 3 * j + a, m]
                    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (c, j, a, m, got, ref)


def check_force_rows_central_fd(orc, h=1e-4):
    w, b, X = tiny_batch()
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    scale = np.abs(K[b.n_cfg:]).max()
    for c in range(b.n_cfg):
        for j in range(int(b.cfg_ptr[c]), int(b.cfg_ptr[c + 1])):
            for a in range(3):
                dp = np.zeros((b.n_atoms, 3), dtype=np.complex128)
                dp[j, a] = h
                for m in range(w.M):
                    ref = -(linearised_energy(w, b, X, c, m, dp).real
                            - linearised_energy(w, b, X, c, m, -dp).real) / (2 * h)
                    assert abs(K[b.n_cfg + 3 * j + a, m] - ref) <= 1e-7 * scale


def strained_energy(w, b, X, r, cfg, m, eps):
    """E_c^m under the homogeneous strain eps (complex 3x3), r_p -> (I + eps) r_p:
    delta^2 sum_{i in c} ((d_i + sum_{p of i} J_p . (eps r_p)) . x_m)^zeta, in plain loops."""
    a0, a1 = int(b.cfg_ptr[cfg]), int(b.cfg_ptr[cfg + 1])
    E = 0j
    for i in range(a0, a1):
        d = b.desc[i].astype(np.complex128)
        for p in range(int(b.pair_ptr[i]), int(b.pair_ptr[i + 1])):
            dr = eps @ r[p]
            for a in range(3):
                d = d + b.jac[p, a].astype(np.float64) * dr[a]
        s = 0j
        for k in range(w.D):
            s += d[k] * X[m, k]
        E += s ** w.zeta
    return w.delta ** 2 * E


def check_virial_rows_strain(orc, h=1e-30):
    # W_ab = - dE / d eps_ba by complex step of the strained, linearised energy,
    # for every configuration, component and sparse point (virial reading)
    w, b, X = tiny_batch()
    r = synth.pair_vectors(w, b)
    K = orc.build_virial_rows(b.cfg_ptr, b.desc, b.pair_ptr, b.jac, r, X, w.zeta, w.delta)
    assert K.shape == (9 * b.n_cfg, w.M)
    for c in range(b.n_cfg):
        for a in range(3):
            for bb in range(3):
                eps = np.zeros((3, 3), dtype=np.complex128)
                eps[bb, a] = 1j * h
                for m in range(w.M):
                    ref = -strained_energy(w, b, X, r, c, m, eps).imag / h
                    got = K[9 * c + 3 * a + bb, m]
                    assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (c, a, bb, m, got, ref)


def permuted_batch(b, rng):
    """Relabel atoms inside each configuration; pairs follow their source."""
    perm = np.empty(b.n_atoms, dtype=np.int64)          # new index of old atom
    for c in range(b.n_cfg):
        a0, a1 = int(b.cfg_ptr[c]), int(b.cfg_ptr[c + 1])
        perm[a0:a1] = a0 + rng.permutation(a1 - a0)
    inv = np.argsort(perm)                              # old atom at new index
    cnt = np.diff(b.pair_ptr)[inv]
    pair_ptr = np.zeros(b.n_atoms + 1, dtype=np.int64)
    np.cumsum(cnt, out=pair_ptr[1:])
    order = np.concatenate([np.arange(b.pair_ptr[o], b.pair_ptr[o + 1]) for o in inv])
    return (b.desc[inv], pair_ptr, perm[b.pair_j[order]].astype(np.int32), b.jac[order], perm)


def check_permutation(orc):
    w, b, X = tiny_batch()
    rng = np.random.default_rng(5)
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    desc, pptr, pj, jac, perm = permuted_batch(b, rng)
    K2 = orc.build_knm(b.cfg_ptr, desc, pptr, pj, jac, X, w.zeta, w.delta)
    assert np.allclose(K2[:b.n_cfg], K[:b.n_cfg], rtol=1e-13, atol=1e-16)
    rows = b.n_cfg + 3 * np.repeat(perm, 3) + np.tile(np.arange(3), b.n_atoms)
    assert np.allclose(K2[rows], K[b.n_cfg:], rtol=1e-12, atol=1e-15)


def check_species_blocks(orc, h=1e-30):
    # per-species GP blocks: (i) energy rows by brute force over the centres of
    # species z, (ii) force rows equal to the complex-step derivative of that
    # energy (linearised descriptor), so pairs are masked by their centre,
    # never by their target, (iii) the blocks of all species add up to the
    # species-blind rows, (iv) a species no atom has gives zero rows
    w, b, X = tiny_batch(TINY.with_(n_cfg=3, atoms_lo=2, atoms_hi=5))
    spc = species_of(b)
    assert 0 < spc.sum() < b.n_atoms
    total = np.zeros((b.n_rows, w.M))
    for z in (0, 1):
        K = orc.build_knm_species(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta,
                                  w.delta, spc, z)
        total += K
        zero = np.zeros((b.n_atoms, 3), dtype=np.complex128)
        for c in range(b.n_cfg):
            for m in range(w.M):
                ref = linearised_energy_species(w, b, X, c, m, zero, spc, z).real
                assert abs(K[c, m] - ref) <= 1e-12 * max(1.0, abs(ref))
            for j in range(int(b.cfg_ptr[c]), int(b.cfg_ptr[c + 1])):
                for a in range(3):
                    dr = np.zeros((b.n_atoms, 3), dtype=np.complex128)
                    dr[j, a] = 1j * h
                    for m in range(w.M):
                        ref = -linearised_energy_species(w, b, X, c, m, dr, spc, z).imag / h
                        got = K[b.n_cfg + 3 * j + a, m]
                        assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (z, c, j, a, m)
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    assert np.allclose(total, K, rtol=1e-13, atol=1e-13 * np.abs(K).max())
    K5 = orc.build_knm_species(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta,
                               w.delta, spc, 5)
    assert not K5.any()


def check_predict_species(orc):
    # a species block's prediction: its energies and forces are its rows times
    # c, its local energies vanish on the other species, and the blocks of all
    # species add up to the species-blind prediction
    w, b, X = tiny_batch(TINY.with_(n_cfg=3, atoms_lo=2, atoms_hi=5))
    spc = species_of(b)
    cc = np.random.default_rng(8).standard_normal(w.M)
    tot = [np.zeros(b.n_atoms), np.zeros(b.n_cfg), np.zeros((b.n_atoms, w.D)),
           np.zeros((b.n_atoms, 3))]
    for z in (0, 1):
        e, ec, g, F = orc.predict_species(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, cc,
                                          w.zeta, w.delta, spc, z)
        K = orc.build_knm_species(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta,
                                  w.delta, spc, z)
        Kc = K @ cc
        assert np.allclose(ec, Kc[:b.n_cfg], rtol=1e-12, atol=1e-12)
        assert np.allclose(F.reshape(-1), Kc[b.n_cfg:], rtol=1e-12, atol=1e-12)
        assert not e[spc != z].any() and not g[spc != z].any()
        for t, v in zip(tot, (e, ec, g, F)):
            t += v
    ref = orc.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, cc, w.zeta, w.delta)
    for t, r in zip(tot, ref):
        assert np.allclose(t, r, rtol=1e-12, atol=1e-12 * max(1.0, np.abs(r).max()))


def check_pair_transpose(orc):
    w, b, X = tiny_batch()
    tptr, tpair = orc.pair_transpose(b.pair_ptr, b.pair_j, b.n_atoms)
    for j in range(b.n_atoms):
        brute = [p for p in range(b.n_pairs) if b.pair_j[p] == j]
        assert list(tpair[tptr[j]:tptr[j + 1]]) == brute


def small_fit_problem(seed=3, jitter=1e-8):
    w, b, X = tiny_batch(TINY.with_(n_cfg=6, atoms_lo=3, atoms_hi=7, D=8, M=6), seed=seed)
    return w, b, X, jitter


def check_qr_vs_closed_forms(orc):
    w, b, X, jit = small_fit_problem()
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    Kmm = orc.build_kmm(X, w.zeta, w.delta)
    rng = np.random.default_rng(7)
    y = rng.standard_normal(b.n_rows)
    sig = synth.sigma_rows(w, b.counts)
    c = orc.fit(K, Kmm, y, sig, jit)
    # eq. GP_L with jitter on K_MM, solved here by an SVD-based route
    w2 = 1.0 / sig ** 2
    lhs = Kmm + jit * np.eye(w.M) + K.T @ (w2[:, None] * K)
    ref = np.linalg.pinv(lhs) @ (K.T @ (w2 * y))
    assert np.linalg.norm(c - ref) <= 1e-8 * np.linalg.norm(ref)
    # least squares of the stacked system by SVD (gelsd), not by QR
    L = np.linalg.cholesky(Kmm + jit * np.eye(w.M))
    A = np.vstack([K / sig[:, None], L.T])
    bb = np.concatenate([y / sig, np.zeros(w.M)])
    ref2 = np.linalg.lstsq(A, bb, rcond=None)[0]
    assert np.linalg.norm(c - ref2) <= 1e-10 * np.linalg.norm(ref2)


def check_fold_streamed(orc):
    # Folding the observation rows block by block (an empty and a one-row block
    # included, in two different orders) must give the least-squares solution of
    # the whole stacked system (SVD route), the residual norm of that solution in
    # the corner, a triangular factor whose Gram matrix is that of [A | b], and
    # one solution whatever the block order.
    w, b, X, jit = small_fit_problem(seed=5)
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    Kmm = orc.build_kmm(X, w.zeta, w.delta)
    y = np.random.default_rng(11).standard_normal(b.n_rows)
    sig = synth.sigma_rows(w, b.counts)
    n = b.n_rows
    cuts = [0, 3, 3, 4, n // 2, n]
    blocks = [(cuts[i], cuts[i + 1]) for i in range(len(cuts) - 1)]
    L = np.linalg.cholesky(Kmm + jit * np.eye(w.M))
    A = np.vstack([K / sig[:, None], L.T])
    bb = np.concatenate([y / sig, np.zeros(w.M)])
    ref = np.linalg.lstsq(A, bb, rcond=None)[0]
    rnorm = np.linalg.norm(bb - A @ ref)
    sols = []
    for order in (blocks, blocks[::-1]):
        T = orc.fold_init(Kmm, jit)
        for r0, r1 in order:
            T = orc.fold_rows(T, K[r0:r1], y[r0:r1], sig[r0:r1])
        assert np.all(np.tril(T, -1) == 0.0)
        Ab = np.column_stack([A, bb])
        G = Ab.T @ Ab
        assert np.linalg.norm(T.T @ T - G) <= 1e-12 * np.linalg.norm(G)
        c, res = orc.fold_solve(T)
        assert np.linalg.norm(c - ref) <= 1e-10 * np.linalg.norm(ref)
        assert abs(res - rnorm) <= 1e-9 * rnorm
        sols.append(c)
    assert np.linalg.norm(sols[0] - sols[1]) <= 1e-10 * np.linalg.norm(sols[0])


def check_refine_step(orc):
    # One seminormal step with the exact factor R of A lands on the least-squares
    # solution (SVD route) from any starting c, since c + (A^T A)^-1 A^T (b - A c)
    # = (A^T A)^-1 A^T b; the rows' share is additive over any split into
    # batches; at the solution the observation rows' share equals
    # (K_MM + jitter I) c (the normal equations); and with an approximate R
    # (K perturbed by 1e-3) the steps still converge to that solution.
    w, b, X, jit = small_fit_problem(seed=9, jitter=1e-2)
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    Kmm = orc.build_kmm(X, w.zeta, w.delta)
    rng = np.random.default_rng(13)
    y = rng.standard_normal(b.n_rows)
    sig = synth.sigma_rows(w, b.counts)
    L = np.linalg.cholesky(Kmm + jit * np.eye(w.M))
    A = np.vstack([K / sig[:, None], L.T])
    bb = np.concatenate([y / sig, np.zeros(w.M)])
    ref = np.linalg.lstsq(A, bb, rcond=None)[0]
    R = np.linalg.qr(A, mode="r")
    c0 = rng.standard_normal(w.M)
    n = b.n_rows
    g, rr = orc.refine_rows(K, y, sig, c0)
    g2 = np.zeros(w.M)
    rr2 = 0.0
    for r0, r1 in ((0, 4), (4, 4), (4, n // 2), (n // 2, n)):
        gb, rb = orc.refine_rows(K[r0:r1], y[r0:r1], sig[r0:r1], c0)
        g2 += gb
        rr2 += rb
    assert np.linalg.norm(g2 - g) <= 1e-12 * np.linalg.norm(g)
    assert abs(rr2 - rr) <= 1e-12 * rr
    assert abs(rr - np.sum(((y - K @ c0) / sig) ** 2)) <= 1e-12 * rr
    c1 = orc.refine_solve(R, Kmm, jit, g, c0)
    assert np.linalg.norm(c1 - ref) <= 1e-8 * np.linalg.norm(ref)
    gs, _ = orc.refine_rows(K, y, sig, ref)
    lhs = Kmm @ ref + jit * ref
    assert np.linalg.norm(gs - lhs) <= 1e-8 * np.linalg.norm(lhs)
    Kp = K * (1.0 + 1e-3 * rng.standard_normal(K.shape))
    Rp = np.linalg.qr(np.vstack([Kp / sig[:, None], L.T]), mode="r")
    c = np.zeros(w.M)
    for _ in range(8):
        c = orc.refine_solve(Rp, Kmm, jit, orc.refine_rows(K, y, sig, c)[0], c)
    assert np.linalg.norm(c - ref) <= 1e-8 * np.linalg.norm(ref)


def check_local_rows(orc):
    # Local-property rows of every atom: summed over each configuration they are
    # the energy rows (L-hat sums the local terms), multiplied by c they are the
    # predicted local energies, and a brute-force loop gives each entry.
    w, b, X = tiny_batch()
    idx = np.arange(b.n_atoms)
    KL = orc.build_local_rows(b.desc, X, idx, w.zeta, w.delta)
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    for c in range(b.n_cfg):
        s = KL[b.cfg_ptr[c]:b.cfg_ptr[c + 1]].sum(axis=0)
        assert np.allclose(s, K[c], rtol=1e-13, atol=1e-13 * np.abs(K[c]).max())
    cc = np.random.default_rng(5).standard_normal(w.M)
    e, _, _, _ = orc.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, None, X, cc, w.zeta, w.delta)
    assert np.allclose(KL @ cc, e, rtol=1e-12, atol=1e-12 * np.abs(e).max())
    sel = np.array([b.n_atoms - 1, 0, 2, 2])
    KS = orc.build_local_rows(b.desc, X, sel, w.zeta, w.delta)
    for r, i in enumerate(sel):
        for m in range(w.M):
            p = sum(float(b.desc[i][d]) * float(X[m][d]) for d in range(w.D))
            assert abs(KS[r, m] - w.delta ** 2 * p ** w.zeta) <= 1e-12 * max(1.0, abs(KS[r, m]))


def check_predict_variance(orc):
    # the same variances from the normal-equation matrices solved directly
    # (no triangular factor), and 0 <= var_i <= k(d_i, d_i)
    w, b, X, jit = small_fit_problem(seed=6)
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    Kmm = orc.build_kmm(X, w.zeta, w.delta)
    y = np.random.default_rng(12).standard_normal(b.n_rows)
    sig = synth.sigma_rows(w, b.counts)
    A, bb = orc.design_matrix(K, Kmm, y, sig, jit)
    R = orc.augmented_r(A, bb)[:w.M, :w.M]
    var = orc.predict_variance(b.desc, X, Kmm, jit, R, w.zeta, w.delta)
    desc = b.desc.astype(np.float64)
    ks = w.delta ** 2 * (desc @ X.T) ** w.zeta
    kii = w.delta ** 2 * np.sum(desc * desc, axis=1) ** w.zeta
    P = Kmm + jit * np.eye(w.M)
    Q = P + K.T @ (K / sig[:, None] ** 2)
    ref = kii - np.einsum("im,im->i", ks, np.linalg.solve(P, ks.T).T) \
        + np.einsum("im,im->i", ks, np.linalg.solve(Q, ks.T).T)
    assert np.abs(var - ref).max() <= 1e-9 * kii.max()
    assert np.all(var >= -1e-12 * kii.max()) and np.all(var <= kii * (1 + 1e-12))


def check_predict_variance_full_gp(orc):
    # Full-GP limit: every training atom is a sparse point, each observation is
    # one atom's local property (L-hat = identity) and the jitter is 0.  The
    # projected-process variance must then be the textbook full-GP posterior
    # variance k** - k*^T (K + Sigma)^-1 k*, both at the training atoms and at
    # descriptors outside the training set (where k** - k*^T K^-1 k* > 0, so a
    # form that keeps only the data term is wrong).
    w = TINY.with_(n_cfg=3, atoms_lo=2, atoms_hi=3, D=10, zeta=2, delta=0.9)
    b = synth.generate(w, threads=1)
    X = b.desc.astype(np.float64)
    N = X.shape[0]
    idx = np.arange(N)
    K = orc.build_local_rows(X, X, idx, w.zeta, w.delta)
    Kmm = orc.build_kmm(X, w.zeta, w.delta)
    sig = np.linspace(0.2, 0.5, N)
    y = np.random.default_rng(21).standard_normal(N)
    A, bb = orc.design_matrix(K, Kmm, y, sig, 0.0)
    R = orc.augmented_r(A, bb)[:N, :N]
    rng = np.random.default_rng(22)
    T = rng.standard_normal((5, w.D))
    T /= np.linalg.norm(T, axis=1)[:, None]
    Q = np.vstack([X, T])
    var = orc.predict_variance(Q, X, Kmm, 0.0, R, w.zeta, w.delta)
    # textbook GP posterior variance, kernel entries by explicit loops
    def k(u, v):
        return w.delta ** 2 * float(np.dot(u, v)) ** w.zeta
    Kf = np.array([[k(u, v) for v in X] for u in X])
    ref = []
    for q in Q:
        ks = np.array([k(q, v) for v in X])
        ref.append(k(q, q) - ks @ np.linalg.solve(Kf + np.diag(sig ** 2), ks))
    ref = np.array(ref)
    assert np.all(ref[N:] > 1e-3), "test descriptors must lie outside the training span"
    assert np.abs(var - ref).max() <= 1e-9 * max(1.0, np.abs(ref).max())


def check_cur_leverage(orc):
    # leverage of full column rank D without jitter: the squared row norms of
    # the left singular vectors (SVD route), summing to rank D; a descriptor
    # along a direction no other atom has gets leverage 1 and is picked first;
    # equal weights make the weighted sampling pick the largest uniforms
    rng = np.random.default_rng(13)
    Dm = rng.standard_normal((40, 6))
    Dm[:, 5] = 0.0
    Dm[17] = 0.0
    Dm[17, 5] = 2.5
    idx, lev = orc.cur_select(Dm, 4, 0.0)
    Us, sv, _ = np.linalg.svd(Dm, full_matrices=False)
    ref = np.sum(Us[:, sv > 1e-12 * sv[0]] ** 2, axis=1)
    assert np.allclose(lev, ref, rtol=1e-12, atol=1e-13)
    assert abs(lev.sum() - 6.0) <= 1e-11 and abs(lev[17] - 1.0) <= 1e-12
    assert idx[0] == 17
    top = sorted(range(40), key=lambda i: (-lev[i], i))[:4]
    assert list(idx) == top
    # 39 unit rows, 13 along each axis: every leverage is 1/13
    Eq = np.zeros((39, 3))
    Eq[np.arange(39), np.arange(39) % 3] = 1.0
    u = rng.random(39)
    idx_u, levq = orc.cur_select(Eq, 5, 0.0, u)
    assert np.allclose(levq, 1.0 / 13.0, rtol=1e-13)
    assert list(idx_u) == sorted(range(39), key=lambda i: (-u[i], i))[:5]


SE2B = dict(delta=1.3, theta=0.6, r_cut=4.5, width=1.0)


def check_2b_rows(orc, h=1e-30):
    # force rows: complex-step derivative of the energy rows' pair sum under
    # atom displacements (pair vectors move by d_j - d_i); pairs past the cutoff
    # give nothing; K_MM symmetric with diagonal delta^2 fc(x)^2; predict = rows . c
    w, b, X = tiny_batch()
    r = synth.pair_vectors(w, b)
    x = synth.sparse_distances(w, 7)
    K = orc.build_2b_rows(b.cfg_ptr, b.pair_ptr, b.pair_j, r, x, **SE2B)
    src = np.repeat(np.arange(b.n_atoms), np.diff(b.pair_ptr))
    rn = np.linalg.norm(r, axis=1)
    assert np.any(rn >= SE2B["r_cut"]) and np.any((rn > 3.5) & (rn < 4.5))
    for a in range(b.n_atoms):
        c = int(np.searchsorted(b.cfg_ptr, a, side="right") - 1)
        for al in range(3):
            e = np.zeros((b.n_atoms, 3), dtype=np.complex128)
            e[a, al] = 1j * h
            for m in range(len(x)):
                E = 0j
                for p in range(int(b.pair_ptr[b.cfg_ptr[c]]), int(b.pair_ptr[b.cfg_ptr[c + 1]])):
                    v = r[p] + e[int(b.pair_j[p])] - e[src[p]]
                    rr = np.sqrt(np.sum(v * v))
                    d2 = SE2B["delta"] ** 2
                    fc = orc.cutoff_fn(rr, SE2B["r_cut"], SE2B["width"])
                    fx = 1.0 if x[m] < SE2B["r_cut"] - SE2B["width"] else \
                        0.5 * (np.cos(np.pi * (x[m] - SE2B["r_cut"] + SE2B["width"]) / SE2B["width"]) + 1)
                    fx = 0.0 if x[m] >= SE2B["r_cut"] else fx
                    E += 0.5 * d2 * fc * fx * np.exp(-(rr - x[m]) ** 2 / (2 * SE2B["theta"] ** 2))
                ref = -E.imag / h
                got = K[b.n_cfg + 3 * a + al, m]
                assert abs(got - ref) <= 1e-12 * max(1.0, abs(ref)), (a, al, m, got, ref)
    rc, wd = SE2B["r_cut"], SE2B["width"]
    fcv = orc.cutoff_fn(np.array([rc - wd - 1e-9, rc - 0.75 * wd, rc - 0.5 * wd, rc - 0.25 * wd,
                                  rc, rc + 1.0]), rc, wd)
    s2 = 0.5 * np.sqrt(2.0)
    assert np.allclose(fcv, [1.0, 0.5 + 0.5 * s2, 0.5, 0.5 - 0.5 * s2, 0.0, 0.0], atol=1e-12)
    Kmm = orc.build_kmm_2b(x, **SE2B)
    assert np.array_equal(Kmm, Kmm.T)
    fx = orc.cutoff_fn(x, SE2B["r_cut"], SE2B["width"])
    assert np.allclose(np.diag(Kmm), SE2B["delta"] ** 2 * fx ** 2, rtol=1e-14)
    cc = np.random.default_rng(8).standard_normal(len(x))
    E, F = orc.predict_2b(b.cfg_ptr, b.pair_ptr, b.pair_j, r, x, cc, **SE2B)
    assert np.allclose(E, K[:b.n_cfg] @ cc, rtol=1e-12, atol=1e-14)
    assert np.allclose(F.reshape(-1), K[b.n_cfg:] @ cc, rtol=1e-12, atol=1e-14)
    # a pair moved past the cutoff drops out of its configuration's energy row
    r2 = r.copy()
    r2[0] *= (SE2B["r_cut"] + 0.1) / np.linalg.norm(r2[0])
    K2 = orc.build_2b_rows(b.cfg_ptr, b.pair_ptr, b.pair_j, r2, x, **SE2B)
    c0 = int(np.searchsorted(b.cfg_ptr, src[0], side="right") - 1)
    drop = 0.5 * orc.se2b_kernel(np.linalg.norm(r[0]), x, **SE2B)
    assert np.allclose(K2[c0], K[c0] - drop, rtol=1e-12, atol=1e-14)


def check_full_gpr_identity(orc):
    # energy-only observations, sparse set = every atom, no jitter:
    # c = L^T (L K L^T + Sigma)^-1 y  (push-through identity of eq. GP_L)
    w = TINY.with_(n_cfg=5, atoms_lo=2, atoms_hi=4, D=12, zeta=2, delta=0.7)
    b = synth.generate(w, threads=1)
    X = b.desc.astype(np.float64)
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    KE = K[:b.n_cfg]
    Kmm = orc.build_kmm(X, w.zeta, w.delta)
    sig = np.full(b.n_cfg, 0.05)
    y = np.random.default_rng(2).standard_normal(b.n_cfg)
    c = orc.fit(KE, Kmm, y, sig, 0.0)
    Lhat = np.zeros((b.n_cfg, b.n_atoms))
    for k in range(b.n_cfg):
        Lhat[k, b.cfg_ptr[k]:b.cfg_ptr[k + 1]] = 1.0
    Kfull = np.array([[w.delta ** 2 * np.dot(p, q) ** w.zeta for q in X] for p in X])
    alpha = np.linalg.solve(Lhat @ Kfull @ Lhat.T + np.diag(sig ** 2), y)
    ref = Lhat.T @ alpha
    assert np.linalg.norm(c - ref) <= 1e-7 * np.linalg.norm(ref)


def check_delta_scaling(orc):
    # K scales with delta^2; scaling Sigma and the jitter by delta^2 as well
    # leaves the posterior mean unchanged and divides c by delta^2.
    w, b, X, jit = small_fit_problem(seed=4)
    y = np.random.default_rng(9).standard_normal(b.n_rows)
    sig = synth.sigma_rows(w, b.counts)
    out = []
    for dl in (1.0, 2.5):
        K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, dl)
        Kmm = orc.build_kmm(X, w.zeta, dl)
        out.append(orc.fit(K, Kmm, y, sig * dl, jit * dl * dl))
    assert np.allclose(out[1] * 2.5 ** 2, out[0], rtol=1e-8, atol=1e-10)


def check_predict_energy_and_gradient(orc, h=1e-30):
    w, b, X = tiny_batch()
    c = np.random.default_rng(3).standard_normal(w.M)
    e, ecfg, g, F = orc.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, c, w.zeta, w.delta)
    for i in range(b.n_atoms):
        ref = sum(c[m] * w.delta ** 2 * np.dot(b.desc[i], X[m]) ** w.zeta for m in range(w.M))
        assert abs(e[i] - ref) <= 1e-13 * max(1, abs(ref))
        # Euler: eps is homogeneous of degree zeta in d_i
        assert abs(np.dot(b.desc[i], g[i]) - w.zeta * e[i]) <= 1e-12 * max(1, abs(e[i]))
        for k in range(w.D):
            d = b.desc[i].astype(np.complex128)
            d[k] += 1j * h
            ref = sum(c[m] * w.delta ** 2 * np.dot(d, X[m]) ** w.zeta for m in range(w.M)).imag / h
            assert abs(g[i, k] - ref) <= 1e-12 * max(1, abs(ref))
    for k in range(b.n_cfg):
        assert abs(ecfg[k] - e[b.cfg_ptr[k]:b.cfg_ptr[k + 1]].sum()) <= 1e-13 * max(1, abs(ecfg[k]))


def check_predict_forces(orc, h=1e-30):
    w, b, X = tiny_batch()
    c = np.random.default_rng(4).standard_normal(w.M)
    _, _, _, F = orc.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, c, w.zeta, w.delta)
    for cfg in range(b.n_cfg):
        for j in range(int(b.cfg_ptr[cfg]), int(b.cfg_ptr[cfg + 1])):
            for a in range(3):
                dr = np.zeros((b.n_atoms, 3), dtype=np.complex128)
                dr[j, a] = 1j * h
                E = sum(c[m] * linearised_energy(w, b, X, cfg, m, dr) for m in range(w.M))
                ref = -E.imag / h
                assert abs(F[j, a] - ref) <= 1e-12 * max(1, abs(ref)), (j, a, F[j, a], ref)


def check_predict_matches_knm(orc):
    # two routes to the same observables: K_NM c and predict
    w, b, X = tiny_batch()
    c = np.random.default_rng(6).standard_normal(w.M)
    K = orc.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    _, ecfg, _, F = orc.predict(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, c, w.zeta, w.delta)
    y = K @ c
    assert np.allclose(y[:b.n_cfg], ecfg, rtol=1e-12, atol=1e-14)
    assert np.allclose(y[b.n_cfg:], F.reshape(-1), rtol=1e-11, atol=1e-14)


def check_backward(orc, h=1e-30):
    w, b, X = tiny_batch()
    rng = np.random.default_rng(8)
    c = rng.standard_normal(w.M)
    ge = rng.standard_normal(b.n_atoms)
    dD, dc, dX = orc.predict_backward(b.desc, X, c, ge, w.zeta, w.delta)

    def L(desc, X_, c_):
        tot = 0j
        for i in range(desc.shape[0]):
            for m in range(X_.shape[0]):
                tot += ge[i] * c_[m] * w.delta ** 2 * np.dot(desc[i], X_[m]) ** w.zeta
        return tot

    L0 = L(b.desc, X, c).real
    # homogeneity: degree 1 in c, degree zeta in X and in desc
    assert abs(np.dot(c, dc) - L0) <= 1e-12 * max(1, abs(L0))
    assert abs(np.sum(X * dX) - w.zeta * L0) <= 1e-11 * max(1, abs(L0))
    assert abs(np.sum(b.desc * dD) - w.zeta * L0) <= 1e-11 * max(1, abs(L0))
    for (arr, grad) in ((b.desc, dD), (X, dX)):
        for idx in [(0, 0), (1, 2), (arr.shape[0] - 1, arr.shape[1] - 1)]:
            A = arr.astype(np.complex128)
            A[idx] += 1j * h
            ref = (L(A, X, c) if arr is b.desc else L(b.desc, A, c)).imag / h
            assert abs(grad[idx] - ref) <= 1e-12 * max(1, abs(ref))
    for m in range(w.M):
        cc = c.astype(np.complex128)
        cc[m] += 1j * h
        ref = L(b.desc, X, cc).imag / h
        assert abs(dc[m] - ref) <= 1e-12 * max(1, abs(ref))


ALL_CHECKS = [check_kmm, check_energy_rows_zeta1, check_energy_rows_zeta2,
              check_energy_rows_bruteforce, check_sparse_self_entry,
              check_force_rows_complex_step, check_force_rows_central_fd,
              check_permutation, check_species_blocks, check_predict_species, check_pair_transpose, check_qr_vs_closed_forms,
              check_fold_streamed, check_refine_step, check_local_rows, check_virial_rows_strain,
              check_predict_variance, check_predict_variance_full_gp, check_cur_leverage, check_2b_rows,
              check_full_gpr_identity, check_delta_scaling,
              check_predict_energy_and_gradient, check_predict_forces,
              check_predict_matches_knm, check_backward]
