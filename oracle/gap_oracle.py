"""Plain, slow, obviously correct FP64 CPU oracle for sparse-GPR GAP fitting.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import this module.
It shares no code, tables or helpers with the GPU library; the two meet only
through arrays produced by the seeded generator in ``synth``.

Everything is computed in float64 with NumPy/SciPy: a library GEMM, Cholesky or
LAPACK QR is used as a single step where the paper's definition calls for that
operation, and nothing is blocked, fused or reordered beyond the definitions
cited on each function (section / equation names of Klawohn et al., "Gaussian
Approximation Potentials: theory, software implementation and application
examples", arXiv:2310.03921).

Notation: descriptors d_i (rows of ``desc``), sparse points x_m (rows of ``X``),
p_im = d_i . x_m, polynomial dot-product kernel k = delta^2 p^zeta,
configuration c with atoms cfg_ptr[c]:cfg_ptr[c+1], neighbour pair (i, k) with
target atom j(i, k) = pair_j[pair_ptr[i] + k] and Jacobian slot
J[pair, alpha, :] = d(d_i)/d(r_{j(i,k), alpha}).
Observation rows: n_cfg total energies first, then 3 force components per atom
in atom-major order (row n_cfg + 3 j + alpha).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack


def _check_zeta(zeta):
    # The dot product of two descriptors may be negative; only an integer
    # exponent >= 1 gives a real kernel there (reading of the dot-product kernel).
    if int(zeta) != zeta or zeta < 1:
        raise ValueError("zeta must be an integer >= 1")
    return int(zeta)


def poly_kernel(p, zeta, delta):
    """k(x, x') = delta^2 (x . x')^zeta.

    Sec. "Regression" (polynomial / dot-product kernel); delta is the
    energy_scale of the GAP string (the GP standard deviation), entering as
    delta^2 on every covariance.
    """
    zeta = _check_zeta(zeta)
    return delta * delta * np.asarray(p, dtype=np.float64) ** zeta


def poly_kernel_grad_scale(p, zeta, delta):
    """d k / d p = delta^2 zeta p^(zeta - 1)  (gradient of the dot-product kernel)."""
    zeta = _check_zeta(zeta)
    return delta * delta * zeta * np.asarray(p, dtype=np.float64) ** (zeta - 1)


def build_kmm(X, zeta, delta):
    """K_MM[m, m'] = k(x_m, x_m')  (Sec. "Theory", definition after eq. GP_L)."""
    X = np.asarray(X, dtype=np.float64)
    return poly_kernel(X @ X.T, zeta, delta)


def pair_transpose(pair_ptr, pair_j, n_atoms):
    """Target-major view of the pair list.

    The operator L-hat (Sec. "Theory") accumulates, for a force observation on
    atom j, every (i, k) pair whose neighbour slot points at j.  Returns
    tgt_ptr [n_atoms+1] and tgt_pair [n_pairs]: pairs pointing at j are
    tgt_pair[tgt_ptr[j]:tgt_ptr[j+1]] in increasing pair order.
    """
    pair_j = np.asarray(pair_j, dtype=np.int64)
    counts = np.bincount(pair_j, minlength=n_atoms)
    tgt_ptr = np.zeros(n_atoms + 1, dtype=np.int64)
    np.cumsum(counts, out=tgt_ptr[1:])
    tgt_pair = np.argsort(pair_j, kind="stable").astype(np.int32)
    return tgt_ptr, tgt_pair


def pair_sources(pair_ptr):
    """Source atom i of every pair (i, k) from the source-major CSR."""
    pair_ptr = np.asarray(pair_ptr, dtype=np.int64)
    return np.repeat(np.arange(len(pair_ptr) - 1), np.diff(pair_ptr))


def build_knm(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta):
    """L-hat K_NM: energy rows then force rows, (n_cfg + 3 N_at) x M, FP64.

    Energy row of configuration c (eq. 1 and eq. epsilon summed by L-hat):
        K_E[c, m] = sum_{i in c} k(d_i, x_m).
    Force row of atom j, component alpha (Sec. "Theory": the derivative rows of
    K_NM are -grad_x k(x_n, x_m) . dx_n/dr_{j alpha}, accumulated by L-hat):
        K_F[(j, alpha), m] = - sum_{(i,k): j(i,k)=j} dk/dp(p_im) (J[(i,k), alpha] . x_m).
    Pairs never leave their configuration, so the sum runs per configuration:
    a GEMM J_c X^T, the elementwise kernel-gradient scale of the source atom,
    and a dense 0/1 incidence matrix (target x pair) for the accumulation.
    """
    cfg_ptr = np.asarray(cfg_ptr, dtype=np.int64)
    pair_ptr = np.asarray(pair_ptr, dtype=np.int64)
    pair_j = np.asarray(pair_j, dtype=np.int64)
    X = np.asarray(X, dtype=np.float64)
    n_cfg, n_at, M = len(cfg_ptr) - 1, int(cfg_ptr[-1]), X.shape[0]
    D = X.shape[1]
    K = np.zeros((n_cfg + 3 * n_at, M))
    for c in range(n_cfg):
        a0, a1 = int(cfg_ptr[c]), int(cfg_ptr[c + 1])
        if a1 == a0:
            continue
        d = np.asarray(desc[a0:a1], dtype=np.float64)
        P = d @ X.T                                          # p_im
        K[c] = poly_kernel(P, zeta, delta).sum(axis=0)
        p0, p1 = int(pair_ptr[a0]), int(pair_ptr[a1])
        if p1 == p0:
            continue
        src = pair_sources(pair_ptr[a0:a1 + 1] - p0)         # local source atom
        tgt = pair_j[p0:p1] - a0                             # local target atom
        if tgt.min() < 0 or tgt.max() >= a1 - a0:
            raise ValueError("a neighbour pair leaves its configuration")
        Jc = np.asarray(jac[p0:p1], dtype=np.float64).reshape(-1, D)
        G = (Jc @ X.T).reshape(p1 - p0, 3, M)                # J[(i,k),alpha] . x_m
        H = poly_kernel_grad_scale(P, zeta, delta)[src][:, None, :] * G
        inc = np.zeros((a1 - a0, p1 - p0))
        inc[tgt, np.arange(p1 - p0)] = 1.0
        KF = -(inc @ H.reshape(p1 - p0, 3 * M)).reshape(a1 - a0, 3, M)
        K[n_cfg + 3 * a0:n_cfg + 3 * a1] = KF.reshape(3 * (a1 - a0), M)
    return K


def build_knm_species(cfg_ptr, desc, pair_ptr, pair_j, jac, X, zeta, delta, species, z):
    """Rows of the per-species GP of species z: L-hat K_NM with only the atoms
    of species z as centres of local energies.

    Sec. "Theory", eq. 1: the energy is a sum over descriptor types of local
    energies, each descriptor type with a GP of its own; a descriptor defined
    for one central species contributes the local energies of the atoms of that
    species only.  With s_i the species of atom i:
        K_E[c, m] = sum_{i in c, s_i = z} k(d_i, x_m)
        K_F[(j, alpha), m] = - sum_{(i,k): j(i,k)=j, s_i = z} dk/dp(p_im) (J[(i,k), alpha] . x_m)
    (targets j of any species).  Computed per configuration as build_knm, the
    kernel values and gradient scales of the other species' centres set to 0.
    """
    cfg_ptr = np.asarray(cfg_ptr, dtype=np.int64)
    pair_ptr = np.asarray(pair_ptr, dtype=np.int64)
    pair_j = np.asarray(pair_j, dtype=np.int64)
    species = np.asarray(species)
    X = np.asarray(X, dtype=np.float64)
    n_cfg, n_at, M = len(cfg_ptr) - 1, int(cfg_ptr[-1]), X.shape[0]
    D = X.shape[1]
    K = np.zeros((n_cfg + 3 * n_at, M))
    for c in range(n_cfg):
        a0, a1 = int(cfg_ptr[c]), int(cfg_ptr[c + 1])
        if a1 == a0:
            continue
        centre = (species[a0:a1] == z).astype(np.float64)[:, None]   # 1 for species z
        d = np.asarray(desc[a0:a1], dtype=np.float64)
        P = d @ X.T
        K[c] = (centre * poly_kernel(P, zeta, delta)).sum(axis=0)
        p0, p1 = int(pair_ptr[a0]), int(pair_ptr[a1])
        if p1 == p0:
            continue
        src = pair_sources(pair_ptr[a0:a1 + 1] - p0)
        tgt = pair_j[p0:p1] - a0
        if tgt.min() < 0 or tgt.max() >= a1 - a0:
            raise ValueError("a neighbour pair leaves its configuration")
        Jc = np.asarray(jac[p0:p1], dtype=np.float64).reshape(-1, D)
        G = (Jc @ X.T).reshape(p1 - p0, 3, M)
        scale = centre * poly_kernel_grad_scale(P, zeta, delta)
        H = scale[src][:, None, :] * G
        inc = np.zeros((a1 - a0, p1 - p0))
        inc[tgt, np.arange(p1 - p0)] = 1.0
        KF = -(inc @ H.reshape(p1 - p0, 3 * M)).reshape(a1 - a0, 3, M)
        K[n_cfg + 3 * a0:n_cfg + 3 * a1] = KF.reshape(3 * (a1 - a0), M)
    return K


def predict_species(cfg_ptr, desc, pair_ptr, pair_j, jac, X, c, zeta, delta, species, z):
    """Prediction of the per-species GP of species z (eq. epsilon for the
    atoms of species z, local energy 0 for the others), with the configuration
    energies, descriptor gradients and forces that follow from those local
    energies by the chain rule."""
    desc = np.asarray(desc, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    centre = (np.asarray(species) == z).astype(np.float64)
    P = desc @ X.T
    e_atom = centre * (poly_kernel(P, zeta, delta) @ c)
    g = centre[:, None] * ((poly_kernel_grad_scale(P, zeta, delta) * c[None, :]) @ X)
    cfg_ptr = np.asarray(cfg_ptr, dtype=np.int64)
    e_cfg = np.array([e_atom[cfg_ptr[k]:cfg_ptr[k + 1]].sum() for k in range(len(cfg_ptr) - 1)])
    forces = None
    if jac is not None:
        src = pair_sources(pair_ptr)
        pj = np.asarray(pair_j, dtype=np.int64)
        forces = np.zeros((desc.shape[0], 3))
        Jp = np.asarray(jac, dtype=np.float64)
        np.add.at(forces, pj, -np.einsum("pad,pd->pa", Jp, g[src]))
    return e_atom, e_cfg, g, forces


def build_virial_rows(cfg_ptr, desc, pair_ptr, jac, pair_r, X, zeta, delta):
    """Virial rows: row 9 c + 3 alpha + beta, column m is
    - sum over the pairs p = (i, k) of configuration c of
      r_p[alpha] * dk/dr_j(p),beta  with  dk/dr_j,beta = delta^2 zeta p_im^(zeta-1) J[p, beta] . x_m.

    Sec. "Theory": virial stresses are sums of partial derivatives of local
    energies; the strain form (r_p -> (I + eps) r_p, W = - dE/d eps^T) is the
    reading taken where the paper gives no formula.
    """
    desc = np.asarray(desc, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    jac = np.asarray(jac, dtype=np.float64)
    r = np.asarray(pair_r, dtype=np.float64)
    S = poly_kernel_grad_scale(desc @ X.T, zeta, delta)
    src = pair_sources(pair_ptr)
    n_cfg = len(cfg_ptr) - 1
    atom_cfg = np.repeat(np.arange(n_cfg), np.diff(np.asarray(cfg_ptr)))
    K = np.zeros((9 * n_cfg, X.shape[0]))
    for p in range(len(src)):
        i = src[p]
        G = jac[p] @ X.T                      # [3 (beta), M]
        c = atom_cfg[i]
        for a in range(3):
            for b in range(3):
                K[9 * c + 3 * a + b] -= r[p, a] * S[i] * G[b]
    return K


def build_local_rows(desc, X, atom_idx, zeta, delta):
    """Rows of local-property observations: row r is k(d_i, x_m), i = atom_idx[r].

    Sec. "Local Property": a per-atom property is learned directly, a mask
    selecting the atoms that carry one, so L-hat of such an observation picks
    one atom's kernel row instead of summing a configuration.
    """
    D = np.asarray(desc, dtype=np.float64)[np.asarray(atom_idx, dtype=np.int64)]
    return poly_kernel(D @ np.asarray(X, dtype=np.float64).T, zeta, delta)


def cur_leverage(desc, jitter):
    """Leverage scores of the data points for CUR selection:
    l_i = d_i^T (D^T D + jitter I)^-1 d_i.

    Sec. "Sparse point selection" (cur_points, after Mahoney & Drineas): the
    column choice of CUR rests on leverage scores; the rank parameter is taken
    as the full rank of the descriptor matrix D (reading), regularised by jitter.
    """
    Dm = np.asarray(desc, dtype=np.float64)
    G = Dm.T @ Dm + jitter * np.eye(Dm.shape[1])
    return np.einsum("ij,ij->i", Dm, np.linalg.solve(G, Dm.T).T)


def cur_select(desc, n_sparse, jitter, u=None):
    """The n_sparse atoms of largest leverage (u None), or exact-size weighted
    sampling without replacement with weights l_i and uniforms u (keys
    log(u_i) / l_i, largest first; Efraimidis & Spirakis).  Ties go to the
    smaller index.  Returns (indices in decreasing key order, leverage)."""
    lev = cur_leverage(desc, jitter)
    if u is None:
        key = lev.copy()
    else:
        with np.errstate(divide="ignore", invalid="ignore"):
            key = np.where(lev > 0, np.log(np.asarray(u, dtype=np.float64)) / lev, -np.inf)
    key = np.where(np.isnan(key), -np.inf, key)
    order = np.lexsort((np.arange(len(key)), -key))
    return order[:n_sparse].astype(np.int64), lev


def cutoff_fn(r, r_cut, width):
    """Cosine cutoff of Sec. "Descriptors based on interatomic distances": 1
    below r_cut - width, 0 from r_cut on, (cos(pi (r - r_cut + width) / width) + 1) / 2
    between (complex arguments branch on their real part)."""
    rr = np.real(r)
    mid = 0.5 * (np.cos(np.pi * (r - r_cut + width) / width) + 1.0)
    return np.where(rr >= r_cut, 0.0, np.where(rr < r_cut - width, 1.0, mid))


def se2b_kernel(r, x, delta, theta, r_cut, width):
    """k(r, x) = delta^2 f_cut(r) f_cut(x) exp(-(r - x)^2 / (2 theta^2)):
    k_SE of Sec. "Regression" on a one-dimensional (distance) descriptor, times
    the cutoff of each distance."""
    return (delta ** 2 * cutoff_fn(r, r_cut, width) * cutoff_fn(x, r_cut, width)
            * np.exp(-(r - x) ** 2 / (2.0 * theta ** 2)))


def se2b_kernel_dr(r, x, delta, theta, r_cut, width):
    """dk/dr of se2b_kernel (r real)."""
    rr = np.asarray(r, dtype=np.float64)
    trans = (rr >= r_cut - width) & (rr < r_cut)
    dfc = np.where(trans, -0.5 * np.pi / width * np.sin(np.pi * (rr - r_cut + width) / width), 0.0)
    e = delta ** 2 * cutoff_fn(x, r_cut, width) * np.exp(-(rr - x) ** 2 / (2.0 * theta ** 2))
    return e * (dfc - cutoff_fn(rr, r_cut, width) * (rr - x) / theta ** 2)


def build_2b_rows(cfg_ptr, pair_ptr, pair_j, pair_r, x, delta, theta, r_cut, width):
    """Rows of a two-body descriptor (energies, then 3 per atom), each directed
    pair p = (i, k) an instance with r = |pair_r[p]| carrying half of its bond:
    energy row c: sum_{p in c} k(r_p, x_m) / 2; force row (a, alpha): minus the
    derivative of that sum by r_a,alpha (r_p = |r_j - r_i|).
    Sec. "Descriptors based on interatomic distances" (distance_2b, cutoff)."""
    x = np.asarray(x, dtype=np.float64)
    R = np.asarray(pair_r, dtype=np.float64)
    src = pair_sources(pair_ptr)
    n_cfg = len(cfg_ptr) - 1
    N = len(pair_ptr) - 1
    atom_cfg = np.repeat(np.arange(n_cfg), np.diff(np.asarray(cfg_ptr)))
    K = np.zeros((n_cfg + 3 * N, len(x)))
    for p in range(len(src)):
        i, j = int(src[p]), int(pair_j[p])
        r = float(np.linalg.norm(R[p]))
        K[atom_cfg[i]] += 0.5 * se2b_kernel(r, x, delta, theta, r_cut, width)
        if r > 0.0:
            dk = se2b_kernel_dr(r, x, delta, theta, r_cut, width)
            u = R[p] / r
            for a in range(3):
                K[n_cfg + 3 * i + a] += 0.5 * dk * u[a]
                K[n_cfg + 3 * j + a] -= 0.5 * dk * u[a]
    return K


def build_kmm_2b(x, delta, theta, r_cut, width):
    x = np.asarray(x, dtype=np.float64)
    return se2b_kernel(x[:, None], x[None, :], delta, theta, r_cut, width)


def predict_2b(cfg_ptr, pair_ptr, pair_j, pair_r, x, c, delta, theta, r_cut, width):
    """Configuration energies and forces of the two-body part with coefficients c."""
    x = np.asarray(x, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    R = np.asarray(pair_r, dtype=np.float64)
    src = pair_sources(pair_ptr)
    n_cfg = len(cfg_ptr) - 1
    N = len(pair_ptr) - 1
    atom_cfg = np.repeat(np.arange(n_cfg), np.diff(np.asarray(cfg_ptr)))
    E = np.zeros(n_cfg)
    F = np.zeros((N, 3))
    for p in range(len(src)):
        i, j = int(src[p]), int(pair_j[p])
        r = float(np.linalg.norm(R[p]))
        E[atom_cfg[i]] += 0.5 * float(se2b_kernel(r, x, delta, theta, r_cut, width) @ c)
        if r > 0.0:
            g = 0.5 * float(se2b_kernel_dr(r, x, delta, theta, r_cut, width) @ c)
            F[i] += g * R[p] / r
            F[j] -= g * R[p] / r
    return E, F


def design_matrix(Knm, Kmm, y, sigma, jitter):
    """A = [Sigma^-1/2 L-hat K_NM ; U_MM], b = [Sigma^-1/2 y ; 0].

    Sec. "Theory": U_MM is the upper Cholesky factor of K_MM after the jitter
    is added to its diagonal (K_MM + jitter I = U^T U).  The padded target is
    scaled by Sigma^-1/2 like the rows of A so that the least-squares problem
    reproduces eq. GP_L (the paper writes b = [y; 0]; this reading is needed
    for the equivalence it states).
    """
    Kmm = np.asarray(Kmm, dtype=np.float64)
    M = Kmm.shape[0]
    U = sla.cholesky(Kmm + jitter * np.eye(M), lower=False)
    w = 1.0 / np.asarray(sigma, dtype=np.float64)
    A = np.vstack([w[:, None] * np.asarray(Knm, dtype=np.float64), U])
    b = np.concatenate([w * np.asarray(y, dtype=np.float64), np.zeros(M)])
    return A, b


def solve_qr(A, b):
    """c = R^-1 Q^T b with A = QR (Householder, LAPACK dgeqrf/dormqr/dtrtrs).

    Sec. "Theory", least-squares form of eq. GP_L solved by QR.
    """
    A = np.asarray(A, dtype=np.float64, order="F")
    n = A.shape[1]
    qr, tau, _, info = lapack.dgeqrf(A)
    if info != 0:
        raise RuntimeError("dgeqrf failed")
    qtb, _, info = lapack.dormqr("L", "T", qr, tau, np.asarray(b, dtype=np.float64)[:, None],
                                 lwork=max(1, 64 * n))
    if info != 0:
        raise RuntimeError("dormqr failed")
    c, info = lapack.dtrtrs(np.triu(qr[:n, :n]), qtb[:n, 0])
    if info != 0:
        raise RuntimeError("R is singular")
    return c


def fit(Knm, Kmm, y, sigma, jitter):
    """Sparse-GPR coefficients by the stable least-squares route (Sec. "Theory")."""
    A, b = design_matrix(Knm, Kmm, y, sigma, jitter)
    return solve_qr(A, b)


def augmented_r(A, b):
    """Upper-triangular factor T of the augmented matrix [A | b] = Q T, (n+1) x (n+1).

    Sec. "Theory", QR route: the first n columns of T are R of A = QR, the last
    holds (Q^T b)[0:n] and, in the corner, the norm of the part of Q^T b that R
    leaves over, i.e. +-||b - A c|| for the least-squares c.  One LAPACK QR of
    [A | b] (zero rows appended when A has fewer than n + 1 rows).
    """
    A = np.asarray(A, dtype=np.float64)
    n = A.shape[1]
    Ab = np.column_stack([A, np.asarray(b, dtype=np.float64)])
    if Ab.shape[0] < n + 1:
        Ab = np.vstack([Ab, np.zeros((n + 1 - Ab.shape[0], n + 1))])
    qr, _, _, info = lapack.dgeqrf(np.asfortranarray(Ab))
    if info != 0:
        raise RuntimeError("dgeqrf failed")
    return np.triu(qr[:n + 1, :n + 1])


def fold_init(Kmm, jitter):
    """State of the streamed fit before any observation: T = [U 0; 0 0].

    The rows U_MM of A with their zero targets (Sec. "Theory"), as an
    (M+1) x (M+1) upper-triangular factor.
    """
    Kmm = np.asarray(Kmm, dtype=np.float64)
    M = Kmm.shape[0]
    T = np.zeros((M + 1, M + 1))
    T[:M, :M] = sla.cholesky(Kmm + jitter * np.eye(M), lower=False)
    return T


def fold_rows(T, Knm_block, y_block, sigma_block):
    """Fold a block of observation rows into the state: T' = factor of [T ; block].

    The block is Sigma^-1/2 [L-hat K_NM | y] of some configurations (rows of A
    and b, Sec. "Theory"); Sec. "Program structure" builds K_NM rows by groups of
    configurations.  Since T^T T is the Gram matrix of the rows seen so far, the
    factor of [T ; block] is that of all rows seen.
    """
    K = np.asarray(Knm_block, dtype=np.float64)
    M = T.shape[0] - 1
    if K.shape[0] == 0:
        return T
    w = 1.0 / np.asarray(sigma_block, dtype=np.float64)
    stacked = np.vstack([T[:, :M], w[:, None] * K])
    rhs = np.concatenate([T[:, M], w * np.asarray(y_block, dtype=np.float64)])
    return augmented_r(stacked, rhs)


def refine_rows(Knm_rows, y, sigma, c):
    """A batch's share of one refinement step of the least-squares fit (Sec.
    "Theory", least-squares form), taken with exact rows.

    With r = Sigma^-1/2 (y - K c) over the batch's rows, returns
    (K^T Sigma^-1/2 r, r . r): summed over all batches, the first is the
    observation rows' part of A^T (b - A c).
    """
    K = np.asarray(Knm_rows, dtype=np.float64)
    w = 1.0 / np.asarray(sigma, dtype=np.float64)
    r = w * (np.asarray(y, dtype=np.float64) - K @ np.asarray(c, dtype=np.float64))
    return K.T @ (w * r), float(r @ r)


def refine_solve(R, Kmm, jitter, g, c):
    """c + dc with R^T R dc = g + U^T (0 - U c), the seminormal correction step.

    g is the observation rows' part of A^T r (refine_rows summed over batches);
    the rows U_MM of A (zero targets) add U^T (0 - U c) = -(K_MM + jitter I) c.
    R is upper triangular M x M, the factor of A or of an approximation of it.
    """
    c = np.asarray(c, dtype=np.float64)
    Kmm = np.asarray(Kmm, dtype=np.float64)
    gt = np.asarray(g, dtype=np.float64) - (Kmm @ c + jitter * c)
    R = np.asarray(R, dtype=np.float64)[:len(c), :len(c)]
    z = sla.solve_triangular(R, gt, trans="T", lower=False)
    return c + sla.solve_triangular(R, z, lower=False)


def fold_solve(T):
    """c = R^-1 (Q^T b)[0:M] and the least-squares residual norm |T[M][M]|."""
    M = T.shape[0] - 1
    c = sla.solve_triangular(T[:M, :M], T[:M, M], lower=False)
    return c, abs(T[M, M])


def solve_normal_equations(Knm, Kmm, y, sigma, jitter):
    """c = [K_MM + K_MN Sigma^-1 K_NM]^-1 K_MN Sigma^-1 y  (eq. GP_L, jitter on K_MM)."""
    Knm = np.asarray(Knm, dtype=np.float64)
    w2 = 1.0 / np.asarray(sigma, dtype=np.float64) ** 2
    M = Knm.shape[1]
    lhs = np.asarray(Kmm) + jitter * np.eye(M) + Knm.T @ (w2[:, None] * Knm)
    rhs = Knm.T @ (w2 * np.asarray(y, dtype=np.float64))
    return np.linalg.solve(lhs, rhs)


def predict(cfg_ptr, desc, pair_ptr, pair_j, jac, X, c, zeta, delta):
    """Local energies, configuration energies, descriptor gradients and forces.

    eq. epsilon: eps_i = sum_m c_m k(d_i, x_m).
    gp_predict gradient: g_i = d eps_i / d d_i = sum_m c_m dk/dp(p_im) x_m.
    Forces by the chain rule (Sec. "Theory"): F_{j alpha} = -dE/dr_{j alpha}
        = - sum_{(i,k): j(i,k)=j} J[(i,k), alpha] . g_i.
    ``jac`` may be None (no forces).
    """
    desc = np.asarray(desc, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    P = desc @ X.T
    e_atom = poly_kernel(P, zeta, delta) @ c
    g = (poly_kernel_grad_scale(P, zeta, delta) * c[None, :]) @ X
    cfg_ptr = np.asarray(cfg_ptr, dtype=np.int64)
    e_cfg = np.array([e_atom[cfg_ptr[k]:cfg_ptr[k + 1]].sum() for k in range(len(cfg_ptr) - 1)])
    forces = None
    if jac is not None:
        n_at = desc.shape[0]
        src = pair_sources(pair_ptr)
        pj = np.asarray(pair_j, dtype=np.int64)
        forces = np.zeros((n_at, 3))
        step = 1 << 16
        for p0 in range(0, len(src), step):
            p1 = min(len(src), p0 + step)
            Jp = np.asarray(jac[p0:p1], dtype=np.float64)
            contrib = np.einsum("pad,pd->pa", Jp, g[src[p0:p1]])
            np.add.at(forces, pj[p0:p1], -contrib)
    return e_atom, e_cfg, g, forces


def predict_variance(desc, X, Kmm, jitter, R, zeta, delta):
    """Predictive variance of the local energies in the sparse GP form of eq. GP_L:
    var_i = k(d_i, d_i) - k_i^T (K_MM + jitter I)^-1 k_i + k_i^T (A^T A)^-1 k_i,
    with A^T A = K_MM + jitter I + K_MN Sigma^-1 K_NM = R^T R, evaluated as
    ||U^-T k_i||^2 and ||R^-T k_i||^2 (U^T U = K_MM + jitter I).

    Sec. "Regression": gp_predict returns the variances the GPR predicts; the
    paper gives no formula, the projected-process form is the reading taken.
    """
    desc = np.asarray(desc, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    M = X.shape[0]
    Kst = poly_kernel(desc @ X.T, zeta, delta)
    kii = poly_kernel(np.einsum("ij,ij->i", desc, desc), zeta, delta)
    U = sla.cholesky(np.asarray(Kmm, dtype=np.float64) + jitter * np.eye(M), lower=False)
    Z1 = sla.solve_triangular(U, Kst.T, trans="T", lower=False)
    Z2 = sla.solve_triangular(np.triu(np.asarray(R, dtype=np.float64)[:M, :M]), Kst.T, trans="T",
                              lower=False)
    return kii - np.sum(Z1 * Z1, axis=0) + np.sum(Z2 * Z2, axis=0)


def predict_backward(desc, X, c, g_e, zeta, delta):
    """Gradients of L = sum_i g_e[i] eps_i with respect to d_i, c and x_m.

    From eq. epsilon with k = delta^2 p^zeta:
      dL/dd_i = g_e[i] sum_m c_m dk/dp(p_im) x_m
      dL/dc_m = sum_i g_e[i] k(p_im)
      dL/dx_m = c_m sum_i g_e[i] dk/dp(p_im) d_i
    """
    desc = np.asarray(desc, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    c = np.asarray(c, dtype=np.float64)
    g_e = np.asarray(g_e, dtype=np.float64)
    P = desc @ X.T
    Sg = poly_kernel_grad_scale(P, zeta, delta)
    d_desc = g_e[:, None] * ((Sg * c[None, :]) @ X)
    d_c = poly_kernel(P, zeta, delta).T @ g_e
    d_X = c[:, None] * ((Sg * g_e[:, None]).T @ desc)
    return d_desc, d_c, d_X
