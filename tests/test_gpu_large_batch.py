"""One whole batch of the 576k-atom mixed-precision fit, in the launch
configuration the benchmark times.

The benchmark cuts the 4000 configurations into batches of about 435,000
observation rows, draws each batch's Jacobians on the device into rows padded
to 128-byte lines, and builds the batch's BF16X3 K_NM rows (L-hat K_NM, Eq. 10
and Eq. 11, energies then forces) straight into the block area of an
M = 8000 FP64 fold state.  This test builds the first such batch the same way
(about 1000 configurations, 142k atoms, 5.7M pairs) and compares the rows of
sampled configurations with the FP64 oracle, which reads the same
device-drawn Jacobians copied back to the host.  Configurations never share
pairs, so each one's rows are self-contained.
"""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu

MIXED_TOL = 1e-4     # split-BF16 contractions vs FP64 oracle
BATCH_ROWS = 435000  # rows per batch, as the benchmark cuts them


def relmax(got, ref):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    return float(np.abs(got - ref).max() / max(np.abs(ref).max(), 1e-300))


@pytest.fixture(scope="module")
def batch():
    import paper_2310_03921_amd as gx
    torch.cuda.set_device(0)
    torch.cuda.empty_cache()
    w = synth.WORKLOADS["fit_large_mixed"]
    counts = synth.atom_counts(w)
    c1 = int(np.searchsorted(np.cumsum(3 * counts + 1), BATCH_ROWS)) + 1
    b = synth.generate(w, np.arange(c1), jac=False)
    ld = synth.jacobian_ld(w.D)
    print(f"\n[large batch] configurations [0, {c1}): {b.n_atoms} atoms, {b.n_pairs} pairs, "
          f"{b.n_rows} rows, Jacobian rows of {ld} floats", flush=True)
    J = torch.zeros(b.n_pairs, 3, ld, dtype=torch.float32, device="cuda")
    synth.device_jacobians(w, 0, c1, out=J)
    atoms = gx.Atoms(torch.tensor(b.cfg_ptr, device="cuda"), torch.tensor(b.desc, device="cuda"),
                     torch.tensor(b.pair_ptr, device="cuda"),
                     torch.tensor(b.pair_j, dtype=torch.int32, device="cuda"), J, w.D)
    X = synth.sparse_points(w)
    sp = gx.Sparse.from_host(X, w.zeta, w.delta)
    gap = gx.Gap(0)
    T = gap.fold_buffer(w.M, b.n_rows)
    gap.build_knm_block(atoms, sp, T, precision="bf16x3")
    torch.cuda.synchronize()
    print("[large batch] rows built", flush=True)
    yield dict(w=w, b=b, X=X, J=J, T=T, c1=c1)
    del atoms, J, T
    torch.cuda.empty_cache()


def test_batch_shape_matches_the_benchmark_cut(batch):
    b, c1 = batch["b"], batch["c1"]
    assert b.n_rows >= BATCH_ROWS > b.n_rows - (3 * int(b.counts[-1]) + 1)
    assert b.n_atoms > 100000 and c1 < synth.WORKLOADS["fit_large_mixed"].n_cfg


def test_sampled_configurations_vs_oracle(batch):
    w, b, X, J, T, c1 = (batch[k] for k in ("w", "b", "X", "J", "T", "c1"))
    M, nc = w.M, b.n_cfg
    cnt = b.counts
    sample = sorted({0, 1, c1 // 2, c1 - 1, int(np.argmax(cnt)), int(np.argmin(cnt))})
    worst = 0.0
    for c in sample:
        a0, a1 = int(b.cfg_ptr[c]), int(b.cfg_ptr[c + 1])
        p0, p1 = int(b.pair_ptr[a0]), int(b.pair_ptr[a1])
        jac = J[p0:p1, :, :w.D].cpu().numpy()
        K = oracle.build_knm(np.array([0, a1 - a0]), b.desc[a0:a1], b.pair_ptr[a0:a1 + 1] - p0,
                             b.pair_j[p0:p1] - a0, jac, X, w.zeta, w.delta)
        rows = np.concatenate([[c], nc + np.arange(3 * a0, 3 * a1)])
        got = T[:M, M + 1 + torch.tensor(rows, device="cuda")].T.cpu().numpy()
        e_e, e_f = relmax(got[:1], K[:1]), relmax(got[1:], K[1:])
        print(f"\nconfiguration {c} ({a1 - a0} atoms): K_E rel {e_e:.2e}, K_F rel {e_f:.2e}",
              flush=True)
        assert e_e <= MIXED_TOL and e_f <= MIXED_TOL, c
        worst = max(worst, e_f)
    assert worst > 0  # split-BF16 rows, not an FP64 path


def test_padding_and_columns_beyond_m_untouched(batch):
    w, b, T = batch["w"], batch["b"], batch["T"]
    M = w.M
    # the state's last column (targets) and rows past the batch are not K_NM rows
    assert torch.count_nonzero(T[M, M + 1:M + 1 + b.n_rows]) == 0
    assert torch.count_nonzero(T[:M, M + 1 + b.n_rows:]) == 0
    assert bool(torch.isfinite(T[:M, M + 1:M + 1 + b.n_rows]).all())
