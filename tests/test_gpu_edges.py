"""Degenerate inputs and argument errors of the added rows and solvers, through
the C ABI: batches without pairs, empty and complete selections, and calls that
the host checks must refuse before any GPU work."""
import ctypes

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


def no_pair_batch(gapx):
    w = synth.Workload("edges", 51, n_cfg=7, atoms_lo=1, atoms_hi=9, D=20, nb=3, M=11)
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    pair_ptr = np.zeros(b.n_atoms + 1, np.int64)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, pair_ptr, np.zeros(0, np.int32), None)
    return w, b, X, atoms


def test_rows_without_pairs(gapx, gap):
    w, b, X, atoms = no_pair_batch(gapx)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    r0 = torch.zeros(0, 3, dtype=torch.float64, device="cuda")
    Kv = gap.build_virial_rows(atoms, sp, r0)
    k2 = gapx.SE2b.from_host(synth.sparse_distances(w, 5), delta=PAR["delta"], theta=PAR["theta"],
                             r_cut=PAR["r_cut"], cut_width=PAR["width"])
    K2 = gap.build_2b_rows(atoms, k2, r0)
    pr = gap.predict_2b(atoms, k2, r0, torch.ones(5, dtype=torch.float64, device="cuda"))
    gap.sync()
    assert torch.all(Kv[:w.M, :9 * b.n_cfg] == 0)
    assert torch.all(K2[:5, :b.n_rows] == 0)
    assert torch.all(pr["e_cfg"] == 0) and torch.all(pr["forces"] == 0)


def test_cur_empty_and_complete_selection(gapx, gap):
    w, b, X, atoms = no_pair_batch(gapx)
    idx0, lev = gap.select_cur(atoms, 0, 1e-8)
    assert idx0.numel() == 0
    idx_all, _ = gap.select_cur(atoms, b.n_atoms, 1e-8)
    assert sorted(idx_all.cpu().tolist()) == list(range(b.n_atoms))
    ref = oracle.cur_leverage(b.desc, 1e-8)
    assert np.abs(lev.cpu().numpy() - ref).max() <= TOL * ref.max()


def test_host_checks_refuse_bad_calls(gapx, gap):
    L = gapx.lib()
    w = synth.Workload("edges", 52, n_cfg=3, atoms_lo=2, atoms_hi=4, D=20, nb=2, M=5)
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    a, s = atoms.struct(), sp.struct()
    out = gapx.colmajor(9 * b.n_cfg + b.n_rows, 8)
    optr = ctypes.c_void_p(out.data_ptr())
    ld = out.shape[1]
    bad = gapx.GAP_E_INVALID
    # pairs but no displacement vectors
    assert L.gap_build_virial_rows(gap._h, ctypes.byref(a), ctypes.byref(s), None, optr, ld) == bad
    assert L.gap_build_virial_rows(gap._h, ctypes.byref(a), ctypes.byref(s),
                                   ctypes.c_void_p(out.data_ptr()), optr, 9 * b.n_cfg - 1) == bad
    # two-body parameters out of range
    x = torch.ones(4, dtype=torch.float64, device="cuda")
    for theta, rc, wd in [(0.0, 4.5, 1.0), (0.5, 4.5, 5.0), (0.5, -1.0, 0.5)]:
        k2 = gapx.gap_se2b(4, x.data_ptr(), 1.0, theta, rc, wd)
        assert L.gap_build_kmm_2b(gap._h, ctypes.byref(k2), optr, ld) == bad
    # selections and sizes
    idx = torch.empty(8, dtype=torch.int32, device="cuda")
    assert L.gap_select_cur(gap._h, ctypes.byref(a), b.n_atoms + 1, 0.0, None,
                            ctypes.c_void_p(idx.data_ptr()), None) == bad
    assert L.gap_select_cur(gap._h, ctypes.byref(a), 1, -1.0, None,
                            ctypes.c_void_p(idx.data_ptr()), None) == bad
    assert L.gap_build_local_rows(gap._h, ctypes.byref(a), ctypes.byref(s), None, 3, optr,
                                  ld) == bad
    var = torch.empty(b.n_atoms, dtype=torch.float64, device="cuda")
    Kmm = gap.build_kmm(sp)
    assert L.gap_predict_variance(gap._h, ctypes.byref(a), ctypes.byref(s),
                                  ctypes.c_void_p(Kmm.data_ptr()), 0.0, None, 8,
                                  ctypes.c_void_p(var.data_ptr())) == bad
    assert L.gap_predict_variance(gap._h, ctypes.byref(a), ctypes.byref(s),
                                  ctypes.c_void_p(Kmm.data_ptr()), 0.0, optr, w.M - 1,
                                  ctypes.c_void_p(var.data_ptr())) == bad
    # the handle still works after the refusals
    gap.sync()
    K = gap.build_knm(atoms, sp)
    ref = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    got = K[:w.M, :b.n_rows].T.cpu().numpy()
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()


def test_fp32_rows_at_an_odd_offset(gapx, gap):
    # FP32 descriptors and Jacobians with D = 252 (rows of 1008 bytes, 16 mod
    # 32): a configuration range starting at an odd atom, and a row slice
    # through the differentiable energy, must reach the ABI as aligned copies
    # and give the oracle's values
    w = synth.Workload("odd32", 61, n_cfg=6, atoms_lo=3, atoms_hi=9, D=252, nb=3, M=17,
                       jac_dtype="f32", desc_dtype="f32")
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    c0 = next(k for k in range(1, b.n_cfg) if b.cfg_ptr[k] % 2 == 1)
    sub = atoms.configs(c0, b.n_cfg)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    K = gap.build_knm(sub, sp)[:w.M, :sub.n_rows].T.cpu().numpy()
    a0, a1 = int(b.cfg_ptr[c0]), int(b.cfg_ptr[-1])
    p0, p1 = int(b.pair_ptr[a0]), int(b.pair_ptr[a1])
    ref = oracle.build_knm(b.cfg_ptr[c0:] - a0, b.desc[a0:a1], b.pair_ptr[a0:a1 + 1] - p0,
                           b.pair_j[p0:p1] - a0, b.jac[p0:p1], X, w.zeta, w.delta)
    assert np.abs(K - ref).max() <= TOL * np.abs(ref).max()
    desc = torch.tensor(b.desc, dtype=torch.float32, device="cuda")[1:]
    Xd = torch.tensor(X, device="cuda")
    c = torch.tensor(np.random.default_rng(3).standard_normal(w.M), device="cuda")
    e = gapx.gap_energy(desc, Xd, c, w.zeta, w.delta).cpu().numpy()
    e_ref = oracle.predict([0, b.n_atoms - 1], b.desc[1:], np.zeros(b.n_atoms, np.int64),
                           np.zeros(0, np.int32), None, X, c.cpu().numpy(), w.zeta, w.delta)[0]
    assert np.abs(e - e_ref).max() <= TOL * np.abs(e_ref).max()
