#!/usr/bin/env python3
"""GAP fit benchmark on one MI355X.

Default (the headline): one step = one whole fit of the largest single-GPU
workload, 4000 configurations of 32-256 atoms (575,746 atoms, 1.73 M
observation rows), D = 1500, 40 neighbours per atom, M = 8000, zeta = 4, FP32
descriptors and Jacobians:
  K_MM -> fold state -> per batch of configurations: Jacobians drawn on the
  device, pair transpose, BF16X3 energy and force rows, fold into the FP64
  Householder QR factor -> back substitution -> FP64 refinement steps (exact
  residual rows, Jacobians drawn again) -> coefficients.
Descriptors, pair lists and targets are resident in HBM before the timed
region; the Jacobians (415 GB) cannot be, so drawing them is part of every
step and is reported separately.  Each step is timed with HIP events on the
stream all work is ordered on.  The JSON line carries the fit time (the
metric), the K_NM assembly rate, the roofline of the dominant kernel (the
BF16X3 force rows) from the library's HIP-event stage timers, the scaled
normal-equation residual of the FP64 system, the FP64 CPU oracle timed on a
bounded sample, and the 116k-atom FP64 fit (D = 252, M = 2000) with its legs.

--workload fit_fp64: the 116k-atom FP64 fit is the headline instead.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GAP fit time (s), K_NM GFLOP/s; mixed vs FP64 at stated force error"
PEAK_FP64_TFLOPS = 78.6     # MI355X dense FP64 matrix
PEAK_BF16_TFLOPS = 2500.0   # MI355X dense BF16 matrix
PEAK_HBM_GBS = 8000.0

# HBM traffic of the dominant kernel of each workload, from two rocprofv3 --pmc
# runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) scaled by what the same
# counters read for a device-to-device copy of known size (FETCH_SIZE x 2.000,
# WRITE_SIZE x 1.000); see profiles/force_rows_fp64_fit_fp64_traffic.md and
# profiles/force_rows_b3w_large_mixed_576k_counters.md.  Reported only while
# the sources that shape the kernel's accesses are the ones that were measured.
TRAFFIC = {
    "fit_fp64": {
        "sources": ['paper_2310_03921_amd/csrc/force_f64.hip', 'paper_2310_03921_amd/csrc/common.h', 'paper_2310_03921_amd/csrc/pairs.hip'],
        "sha256": "445e006a1883154a42414d7a8b5f84c9b7b6aff105ed5a00a18b893e1906b6ec",
        "fetch_kib": 38401973, "fetch_scale": 2.000,
        "write_kib": 17887717, "write_scale": 1.000,
    },
    "fit_large_mixed": {
        "sources": ['paper_2310_03921_amd/csrc/mixed.hip', 'paper_2310_03921_amd/csrc/mma_bf16.h', 'paper_2310_03921_amd/csrc/common.h', 'paper_2310_03921_amd/csrc/pairs.hip'],
        "sha256": "1ec31a79bfc19696a707564d9646bde085707dbfe732a64a0b0062cc3607935a",
        "fetch_kib": 513259633, "fetch_scale": 2.000,
        "write_kib": 55306258, "write_scale": 1.000,
    },
}


def force_traffic_bytes(w):
    """HBM bytes per launch of the workload's force-row kernel, or None."""
    import hashlib
    t = TRAFFIC.get(w.name)
    if t is None:
        return None
    h = hashlib.sha256()
    try:
        for src in t["sources"]:
            with open(os.path.join(ROOT, src), "rb") as f:
                h.update(f.read())
    except OSError:
        return None
    if h.hexdigest() != t["sha256"]:
        return None
    return t["fetch_kib"] * 1024.0 * t["fetch_scale"] + t["write_kib"] * 1024.0 * t["write_scale"]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def describe(w, b):
    return (f"{w.name}: {w.n_cfg} configurations x U[{w.atoms_lo},{w.atoms_hi}] atoms "
            f"({b.n_atoms} atoms, {b.n_pairs} pairs, {b.n_rows} observation rows), D={w.D}, "
            f"{w.nb} neighbours/atom, M={w.M}, zeta={w.zeta}, delta={w.delta}, "
            f"J {w.jac_dtype}")


def host_info():
    """Threads the oracle's BLAS uses, the host's logical CPUs, CPU model and BLAS."""
    info = {"logical_cpus": os.cpu_count()}
    try:
        from threadpoolctl import threadpool_info
        pools = threadpool_info()
        info["blas_threads"] = max([p.get("num_threads", 1) for p in pools] or [1])
        info["blas"] = sorted({f"{p.get('internal_api')} {p.get('version')}" for p in pools
                               if p.get("user_api") == "blas"})
    except Exception:
        info["blas_threads"] = os.cpu_count() or 1
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    info["cpu_model"] = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return info


def cpu_baseline(w, b, X, n_sample):
    """FP64 oracle on the first n_sample configurations of the 116k-atom fit
    (measured parts listed, and their extrapolation to the whole fit)."""
    import oracle
    import synth
    hi = host_info()
    n_sample = min(n_sample, b.n_cfg)
    a1 = int(b.cfg_ptr[n_sample])
    p1 = int(b.pair_ptr[a1])
    t0 = time.perf_counter()
    K = oracle.build_knm(b.cfg_ptr[:n_sample + 1], b.desc[:a1], b.pair_ptr[:a1 + 1],
                         b.pair_j[:p1], b.jac[:p1], X, w.zeta, w.delta)
    t_knm = time.perf_counter() - t0
    t0 = time.perf_counter()
    Kmm = oracle.build_kmm(X, w.zeta, w.delta)
    t_kmm = time.perf_counter() - t0
    y = np.random.default_rng(0).standard_normal(K.shape[0])
    sig = synth.sigma_rows(w, b.counts[:n_sample])
    t0 = time.perf_counter()
    A, bb = oracle.design_matrix(K, Kmm, y, sig, w.jitter)
    t_chol = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.solve_qr(A, bb)
    t_qr = time.perf_counter() - t0
    m_full = b.n_rows + w.M
    est = t_knm * (b.n_cfg / n_sample) + t_kmm + t_chol + t_qr * (m_full / A.shape[0])
    return {"value": est, "unit": "s", "cores": int(hi["blas_threads"]), "kind": "oracle",
            "sample": (f"oracle K_NM on {n_sample} of {b.n_cfg} configurations "
                       f"({t_knm:.2f} s, scaled x{b.n_cfg / n_sample:.1f}); K_MM {t_kmm:.2f} s; "
                       f"Cholesky+stack {t_chol:.2f} s; LAPACK QR of the {A.shape[0]} x {w.M} "
                       f"sampled system ({t_qr:.2f} s, scaled by rows x{m_full / A.shape[0]:.1f})"),
            "measured_s": t_knm + t_kmm + t_chol + t_qr, "extrapolated": True, "host": hi}


def cpu_baseline_full(w, b, X):
    """FP64 oracle on the whole 116k-atom fit: K_NM of every configuration,
    K_MM, the stacked least-squares system and its LAPACK QR solve (no sample)."""
    import oracle
    import synth
    hi = host_info()
    t0 = time.perf_counter()
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    t_knm = time.perf_counter() - t0
    log(f"oracle K_NM of the whole fit: {t_knm:.1f} s")
    t0 = time.perf_counter()
    Kmm = oracle.build_kmm(X, w.zeta, w.delta)
    t_kmm = time.perf_counter() - t0
    y = np.random.default_rng(0).standard_normal(K.shape[0])
    sig = synth.sigma_rows(w, b.counts)
    t0 = time.perf_counter()
    A, bb = oracle.design_matrix(K, Kmm, y, sig, w.jitter)
    del K
    t_chol = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.solve_qr(A, bb)
    t_qr = time.perf_counter() - t0
    log(f"oracle QR of the {A.shape[0]} x {w.M} system: {t_qr:.1f} s")
    tot = t_knm + t_kmm + t_chol + t_qr
    return {"value": tot, "unit": "s", "cores": int(hi["blas_threads"]), "kind": "oracle",
            "sample": (f"whole 116k-atom FP64 fit, not sampled: K_NM {t_knm:.1f} s, K_MM "
                       f"{t_kmm:.2f} s, Cholesky+stack {t_chol:.2f} s, LAPACK QR of the "
                       f"{A.shape[0]} x {w.M} system {t_qr:.1f} s"),
            "measured_s": tot, "extrapolated": False, "host": hi}


def cpu_baseline_large(synth, n_sample=2):
    """FP64 oracle on a bounded sample of the 576k-atom fit, timed, never
    extrapolated (the whole fit would need ~530 GB of host memory): K_NM of its
    first n_sample configurations (Jacobians drawn on the device and copied
    back, outside the timing), K_MM of all 8000 sparse points, and the LAPACK QR
    of the sample's stacked least-squares system."""
    import oracle
    import torch
    hi = host_info()
    w = synth.WORKLOADS["fit_large_mixed"]
    b = synth.generate(w, np.arange(n_sample), jac=False)
    b.jac = synth.device_jacobians(w, 0, n_sample).cpu().numpy()[:, :, :w.D]
    torch.cuda.synchronize()
    X = synth.sparse_points(w)
    t0 = time.perf_counter()
    K = oracle.build_knm(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac, X, w.zeta, w.delta)
    t_knm = time.perf_counter() - t0
    t0 = time.perf_counter()
    Kmm = oracle.build_kmm(X, w.zeta, w.delta)
    t_kmm = time.perf_counter() - t0
    y = np.random.default_rng(0).standard_normal(K.shape[0])
    sig = synth.sigma_rows(w, b.counts)
    t0 = time.perf_counter()
    A, bb = oracle.design_matrix(K, Kmm, y, sig, w.jitter)
    t_chol = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.solve_qr(A, bb)
    t_qr = time.perf_counter() - t0
    tot = t_knm + t_kmm + t_chol + t_qr
    return {"value": tot, "unit": "s", "cores": int(hi["blas_threads"]), "kind": "oracle",
            "sample": (f"{n_sample} of 4000 configurations of the 576k-atom fit ({b.n_atoms} atoms, "
                       f"{b.n_rows} rows): K_NM {t_knm:.2f} s, K_MM (8000 x 8000, D = 1500) "
                       f"{t_kmm:.2f} s, Cholesky+stack {t_chol:.2f} s, LAPACK QR of the "
                       f"{A.shape[0]} x {w.M} sampled system {t_qr:.2f} s; measured, not "
                       f"extrapolated to the whole fit"),
            "measured_s": tot, "extrapolated": False, "host": hi}


def measured_peaks(torch):
    """Dense FP64 and BF16 matrix-core rates of this device, from the probe
    library (independent products, no memory traffic): the measured
    denominators reported beside the spec peaks.  Each is measured twice: on
    constant operands, and on pseudo-random operands that change every product
    (the matrix cores draw more power on those, and under the power limit the
    clock drops; kernels on real data are held to the second figure)."""
    import ctypes
    path = os.path.join(ROOT, "paper_2310_03921_amd", "libgap_peak.so")
    if not os.path.exists(path):
        return None
    L = ctypes.CDLL(path)
    L.gap_peak_mfma.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_int,
                                ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_double)]
    L.gap_peak_mfma.restype = ctypes.c_int
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = 2 * cus                     # two waves per SIMD
    out = torch.empty(blocks * 256, dtype=torch.float64, device="cuda")
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    res = {"cus": cus, "blocks": blocks}
    for kind, name, iters in ((0, "fp64", 200_000), (1, "bf16", 800_000),
                              (3, "fp64_random_operands", 200_000),
                              (2, "bf16_random_operands", 800_000)):
        ms, fl = ctypes.c_double(), ctypes.c_double()
        best = 0.0
        for it in (iters // 20, iters, iters):
            if L.gap_peak_mfma(st, kind, it, blocks, ctypes.c_void_p(out.data_ptr()),
                               ctypes.byref(ms), ctypes.byref(fl)) != 0:
                return None
            best = max(best, fl.value / (ms.value * 1e-3) / 1e12)
        res[name + "_tflops"] = best
    log(f"measured matrix-core peaks: FP64 {res['fp64_tflops']:.1f} TFLOP/s "
        f"({res['fp64_random_operands_tflops']:.1f} on random operands), BF16 "
        f"{res['bf16_tflops']:.0f} TFLOP/s ({res['bf16_random_operands_tflops']:.0f} on random "
        f"operands)")
    return res


class LargeFit:
    """The largest fit (4000 configurations of 32-256 atoms, ~576k atoms, D = 1500,
    40 neighbours, M = 8000, FP32 descriptors and Jacobians, BF16X3 assembly,
    FP64 QR and refinement).  Its 415 GB of Jacobians do not fit in device
    memory, so the configurations are taken in batches of about ``rows``
    observation rows and every pass over the training set draws each batch's
    Jacobians again on the device (counter-based generator, a stand-in for
    the descriptor code that would produce them); a pass starts with the batch
    whose Jacobians the buffer still holds from the pass before, and does not
    draw those again.  One fit:
      K_MM -> fold state [U 0; 0 0] -> per batch: Jacobians, BF16X3 rows (pair
      transpose, split, energy rows + S, force rows) into the state's block
      area, fold (Householder QR of [T; block]) -> back substitution ->
      up to ``refine`` steps, each a pass of exact FP64 residual rows
      (Jacobians drawn again) and a seminormal correction.  The steps stop
      once the error they leave is predicted below ``refine_tol`` (relative to
      c): each step contracts the error by about the same factor, estimated as
      |dc_k| / |dc_k-1|, so the error after step k is about |dc_k|^2 / |dc_k-1|.
    Descriptors, pair lists and targets stay resident between fits."""

    def __init__(self, args, torch, synth, gapx):
        self.torch, self.synth, self.gapx = torch, synth, gapx
        w = synth.WORKLOADS["fit_large_mixed"]
        self.w = w
        n_cfg = min(w.n_cfg, args.large_cfgs) if args.large_cfgs > 0 else w.n_cfg
        self.refine = args.refine_steps
        self.refine_tol = args.refine_tol
        self.steps_taken = []
        t0 = time.perf_counter()
        log(f"large fit: generating descriptors and neighbour lists of {n_cfg} configurations "
            f"on the host")
        b = synth.generate(w, np.arange(n_cfg), jac=False)
        X = synth.sparse_points(w, b if n_cfg == w.n_cfg else None)
        rows = 3 * b.counts + 1
        cuts, acc = [0], 0
        for c in range(n_cfg):
            acc += int(rows[c])
            if acc >= args.large_rows:
                cuts.append(c + 1)
                acc = 0
        if cuts[-1] != n_cfg:
            cuts.append(n_cfg)
        self.n_cfg, self.n_atoms, self.n_pairs = n_cfg, b.n_atoms, b.n_pairs
        self.n_rows = b.n_rows
        torch.cuda.set_device(0)
        self.gap = gapx.Gap(0)
        self.sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
        max_pairs = max(int(b.pair_ptr[b.cfg_ptr[c1]] - b.pair_ptr[b.cfg_ptr[c0]])
                        for c0, c1 in zip(cuts[:-1], cuts[1:]))
        # rows padded to 128-byte lines (zero padding, never read)
        self.J = torch.zeros(max_pairs, 3, self.synth.jacobian_ld(w.D), dtype=torch.float32,
                             device="cuda")
        self.batches = []
        for c0, c1 in zip(cuts[:-1], cuts[1:]):
            a0, a1 = int(b.cfg_ptr[c0]), int(b.cfg_ptr[c1])
            p0, p1 = int(b.pair_ptr[a0]), int(b.pair_ptr[a1])
            at = gapx.Atoms(torch.tensor(b.cfg_ptr[c0:c1 + 1] - a0, device="cuda"),
                            torch.tensor(b.desc[a0:a1], device="cuda"),
                            torch.tensor(b.pair_ptr[a0:a1 + 1] - p0, device="cuda"),
                            torch.tensor(b.pair_j[p0:p1] - a0, dtype=torch.int32, device="cuda"),
                            self.J[:p1 - p0], w.D)
            self.batches.append({"c0": c0, "c1": c1, "atoms": at, "rows": at.n_rows,
                                 "counts": b.counts[c0:c1]})
        del b
        self.max_rows = max(bt["rows"] for bt in self.batches)
        self.T = self.gap.fold_buffer(w.M, self.max_rows)
        # each batch's exact FP64 kernel-gradient scale, formed once per fit and
        # kept for every refinement pass
        ldS = (w.M + 3) // 4 * 4
        for bt in self.batches:
            bt["S"] = torch.empty(bt["atoms"].n_atoms, ldS, dtype=torch.float64, device="cuda")
        self.Kmm = gapx.colmajor(w.M, w.M, w.M)
        self.t_host = time.perf_counter() - t0
        self.gen_events = []
        self.resident = None
        log(f"large fit: {self.n_atoms} atoms, {self.n_pairs} pairs, {self.n_rows} rows in "
            f"{len(self.batches)} batches of <= {self.max_rows} rows; state "
            f"{self.T.numel() * 8 / 1e9:.1f} GB, Jacobian buffer "
            f"{self.J.numel() * 4 / 1e9:.1f} GB; host set-up {self.t_host:.1f} s")
        # targets: FP64 predict with the hidden coefficients plus seeded noise
        cstar = torch.tensor(synth.hidden_coefficients(w), device="cuda")
        ids = np.arange(n_cfg)
        for bt in self.batches:
            self.jacobians(bt)
            pr = self.gap.predict(bt["atoms"], self.sp, cstar, e_atom=False, e_cfg=True,
                                  forces=True)
            y = torch.cat([pr["e_cfg"], pr["forces"].reshape(-1)])
            y += torch.tensor(synth.noise(w, ids[bt["c0"]:bt["c1"]], bt["counts"]), device="cuda")
            bt["y"] = y
            bt["sigma"] = torch.tensor(synth.sigma_rows(w, bt["counts"]), device="cuda")
        torch.cuda.synchronize()
        self.gen_events = []

    def jacobians(self, bt):
        """Draw the batch's Jacobians into the buffer, unless they are the ones
        it already holds."""
        if self.resident is bt:
            return
        ev = (self.torch.cuda.Event(enable_timing=True), self.torch.cuda.Event(enable_timing=True))
        ev[0].record()
        self.synth.device_jacobians(self.w, bt["c0"], bt["c1"], out=self.J)
        ev[1].record()
        self.gen_events.append(ev)
        self.resident = bt

    def pass_order(self):
        """The batches of one pass, the one whose Jacobians are resident first
        (a pass sums over batches, so any order gives the same result up to the
        rounding of that sum)."""
        r = [bt for bt in self.batches if bt is self.resident]
        return r + [bt for bt in self.batches if bt is not self.resident]

    def fit(self, norms=False):
        """One whole fit; returns c (and, with norms, the block norms for the report)."""
        gap, w, sp, T, M = self.gap, self.w, self.sp, self.T, self.w.M
        gap.build_kmm(sp, out=self.Kmm)
        gap.fold_init(T, M, self.Kmm, w.jitter)
        fro2 = 0.0
        for bt in self.pass_order():
            self.jacobians(bt)
            gap.build_knm_block(bt["atoms"], sp, T, precision="bf16x3")
            if norms:
                w2 = bt["sigma"] ** -2
                for c0 in range(0, M, 512):
                    blk = T[c0:min(M, c0 + 512), M + 1:M + 1 + bt["rows"]]
                    fro2 += float(((blk * blk) @ w2).sum())
            gap.fold_rows(T, M, bt["rows"], bt["y"], bt["sigma"])
        c, lsq, rd = gap.fold_solve(T, M)
        if self.refine > 0:
            for bt in self.batches:
                gap.refine_weights(bt["atoms"], sp, out=bt["S"])
        prev, taken = None, 0
        self.step_norms = []
        for _ in range(self.refine):
            g = self.residual_pass(c)
            gap.refine_solve(T, M, self.Kmm, w.jitter, g, c)   # g holds the step dc
            taken += 1
            ng, nc = self.torch.stack([self.torch.linalg.vector_norm(g),
                                       self.torch.linalg.vector_norm(c)]).tolist()
            step = ng / max(nc, 1e-300)
            self.step_norms.append(step)
            if step == 0.0 or (prev is not None and step * step / prev <= self.refine_tol):
                break
            prev = step
        self.steps_taken.append(taken)
        return (c, lsq, rd, fro2) if norms else c

    def residual_pass(self, c, rr=None):
        g = self.torch.zeros(self.w.M, dtype=self.torch.float64, device="cuda")
        for bt in self.pass_order():
            self.jacobians(bt)
            self.gap.refine_rows_s(bt["atoms"], self.sp, bt["S"], c, bt["y"], bt["sigma"], g, rr)
        return g

    def generation_ms(self):
        self.torch.cuda.synchronize()
        t = sum(a.elapsed_time(b) for a, b in self.gen_events)
        self.gen_events = []
        return t

    def describe(self):
        w = self.w
        return (f"fit_large_mixed: {self.n_cfg} configurations x U[{w.atoms_lo},{w.atoms_hi}] atoms "
                f"({self.n_atoms} atoms, {self.n_pairs} pairs, {self.n_rows} observation rows), "
                f"D={w.D}, {w.nb} neighbours/atom, M={w.M}, zeta={w.zeta}, FP32 descriptors and "
                f"Jacobians (drawn on the device in every pass but for the batch still "
                f"resident from the previous one), BF16X3 rows folded in "
                f"{len(self.batches)} batches into an FP64 Householder QR, up to {self.refine} "
                f"FP64 refinement steps (stopping once the predicted error of c is below "
                f"{self.refine_tol:g})")


def large_knm_bench(args, torch, synth, gapx):
    """K_NM assembly alone on the 576k-atom workload: per step, every batch's
    Jacobians drawn and its BF16X3 rows built into the fold state's block area
    (the assembly half of a fit, without folds or refinement)."""
    L = LargeFit(args, torch, synth, gapx)
    gap, M = L.gap, L.w.M
    # a device-to-device copy of known size (every byte read once and written
    # once): a counter run of this mode reads the counters' scale off it
    cal = torch.ones(1 << 29, dtype=torch.float64, device="cuda")
    cal_out = torch.empty_like(cal)
    cal_out.copy_(cal)
    torch.cuda.synchronize()
    log(f"calibration copy of {cal.numel() * 8} bytes")
    del cal, cal_out

    def step():
        for bt in L.batches:
            L.jacobians(bt)
            gap.build_knm_block(bt["atoms"], L.sp, L.T, precision="bf16x3")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    L.generation_ms()
    gap.timing(True)
    gap.timing_read(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for i in range(args.steps):
        step()
        log(f"assembly step {i + 1}/{args.steps} enqueued")
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    gen = L.generation_ms() / args.steps
    st = gap.timing_read(reset=True)
    per = {k: v[0] / args.steps for k, v in st.items() if v[1] > 0}
    D, P = L.w.D, L.n_pairs
    knm_flops = 2.0 * M * D * (L.n_atoms + 3.0 * P)
    out = {"leg": "knm_assembly_large", "workload": L.describe(), "steps": args.steps,
           "assembly_ms": ms, "jacobian_generation_ms": gen,
           "knm_tflops_algorithmic": knm_flops / ((ms - gen) * 1e-3) / 1e12,
           "stage_ms": {k: round(v, 1) for k, v in per.items()}}
    log(f"K_NM assembly {ms:.0f} ms per pass (generation {gen:.0f} ms)")
    gap.close()
    return out


def large_fit_bench(args, torch, synth, gapx):
    """The headline: whole fits of the largest workload, timed end to end with
    HIP events on the stream every call is ordered on."""
    L = LargeFit(args, torch, synth, gapx)
    gap, w, M = L.gap, L.w, L.w.M
    for i in range(args.warmup):
        t0 = time.perf_counter()
        L.fit()
        torch.cuda.synchronize()
        log(f"large warmup {i + 1}/{args.warmup}: {time.perf_counter() - t0:.2f} s")
    L.generation_ms()
    gap.timing(True)
    gap.timing_read(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    times = []
    n_warm = len(L.steps_taken)
    e0.record()
    for i in range(args.steps):
        s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s0.record()
        c = L.fit()
        s1.record()
        s1.synchronize()
        times.append(s0.elapsed_time(s1))
        log(f"large step {i + 1}/{args.steps}: {times[-1] / 1e3:.2f} s")
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    gen_ms = L.generation_ms() / args.steps
    st = gap.timing_read(reset=True)
    gap.timing(False)
    per = {k: v[0] / args.steps for k, v in st.items() if v[1] > 0}
    fit_s = total_ms / args.steps / 1e3
    assert torch.isfinite(c).all().item(), "non-finite coefficients"
    # accuracy report outside the timed region: one more fit with the block norms,
    # and a final pass for r and A^T r of the exact FP64 system
    timed_steps = L.steps_taken[n_warm:n_warm + args.steps]
    c, lsq, rd, fro2_obs = L.fit(norms=True)
    if L.refine == 0:
        for bt in L.batches:
            gap.refine_weights(bt["atoms"], L.sp, out=bt["S"])
    rr = torch.zeros(1, dtype=torch.float64, device="cuda")
    g = L.residual_pass(c, rr)
    Kc = L.Kmm.T @ c + w.jitter * c             # (K_MM + jitter I) c = U^T U c
    atr = g - Kc                                 # A^T r, regulariser rows included
    r2 = float(rr[0]) + float(c @ Kc)            # ||b - A c||^2 (obs rows + ||U c||^2)
    fro2 = fro2_obs + float(torch.trace(L.Kmm)) + M * w.jitter   # ||U||_F^2 = trace(K_MM + jitter I)
    nA, nc = fro2 ** 0.5, float(torch.linalg.vector_norm(c))
    scaled = float(torch.linalg.vector_norm(atr)) / (nA * (nA * nc + r2 ** 0.5))
    L.generation_ms()
    force_ms = per.get("force_rows", float("nan"))
    D, P = w.D, L.n_pairs
    force_flops = 2.0 * 3.0 * P * M * D            # algorithmic, per fit (all batches)
    exec_flops = 3.0 * 2.0 * 3.0 * P * M * ((D + 31) // 32 * 32)
    knm_ms = sum(per.get(k, 0.0) for k in ("pair_transpose", "energy_rows", "force_rows",
                                             "split_bf16"))
    knm_flops = 2.0 * M * D * (L.n_atoms + 3.0 * P)
    qr_ms = per.get("qr_panel", 0.0) + per.get("qr_update", 0.0)
    m_all = L.n_rows + len(L.batches) * (M + 1)
    qr_flops = 2.0 * m_all * (M + 1) ** 2 - len(L.batches) * 2.0 / 3.0 * (M + 1) ** 3
    line = {
        "metric": METRIC, "value": fit_s, "unit": "s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": fit_s * 1e3, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16x3+f64", "data": "synthetic",
        "config": {"workload": L.describe(), "precision": "bf16x3 assembly, fp64 QR/solve/refinement",
                   "n_rows": L.n_rows, "M": M, "D": D},
        "fit_s_per_step": [t / 1e3 for t in times],
        "jacobian_generation_s": gen_ms / 1e3,
        "fit_s_excluding_generation": fit_s - gen_ms / 1e3,
        "knm_ms": knm_ms,
        "knm_gflops_algorithmic": knm_flops / (knm_ms * 1e-3) / 1e9 if knm_ms > 0 else None,
        "qr_ms": qr_ms, "qr_tflops": qr_flops / (qr_ms * 1e-3) / 1e12 if qr_ms > 0 else None,
        "refinement_ms": per.get("refinement", 0.0),
        "refinement_steps_per_fit": timed_steps,
        "refinement_step_norms": L.step_norms,    # |dc| / |c| of each step (report fit)
        "refinement_tol": L.refine_tol,
        "stage_ms": {k: round(v, 1) for k, v in per.items()},
        # algorithmic flops (6 M D per pair) against the peak of the BF16X3 form:
        # three BF16 matrix-core products per multiply-add, so a third of the
        # BF16 peak; the executed rate against the BF16 peak is the same fraction
        "roofline": {"kernel": "k_force_rows_b3w (BF16X3 force observation rows)",
                     "bound": "mfma", "achieved": force_flops / (force_ms * 1e-3) / 1e12,
                     "peak": PEAK_BF16_TFLOPS / 3.0, "unit": "TFLOP/s",
                     "peak_dtype": "bf16x3 (2500 TFLOP/s BF16 dense / 3 products)",
                     "frac": force_flops / (force_ms * 1e-3) / 1e12 / (PEAK_BF16_TFLOPS / 3.0),
                     "traffic": force_traffic_bytes(w), "traffic_unit": "bytes per launch",
                     "flops_per_launch": force_flops / len(L.batches),
                     "launches_per_fit": len(L.batches),
                     "avg_launch_ms": force_ms / len(L.batches),
                     "executed_tflops": exec_flops / (force_ms * 1e-3) / 1e12,
                     "frac_executed_of_bf16_peak":
                         exec_flops / (force_ms * 1e-3) / 1e12 / PEAK_BF16_TFLOPS},
        "accuracy": {"scaled_normal_eq_residual": scaled,
                     "normal_eq_residual": float(torch.linalg.vector_norm(atr)),
                     "lsq_resid_norm_before_refinement": lsq, "resid_norm_after": r2 ** 0.5,
                     "min_max_abs_rdiag": list(rd)},
        "host_setup_s": L.t_host,
    }
    log(f"large fit {fit_s:.2f} s per fit (Jacobian generation {gen_ms / 1e3:.2f} s), force rows "
        f"{force_ms / 1e3:.2f} s ({line['roofline']['frac']:.2f} of BF16 peak executed), QR "
        f"{qr_ms / 1e3:.2f} s, refinement {line['refinement_ms'] / 1e3:.2f} s, scaled "
        f"normal-equation residual {scaled:.2e}")
    gap.close()
    del L
    torch.cuda.empty_cache()
    return line


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="fit_large_mixed", choices=["fit_large_mixed", "fit_fp64"],
                    help="headline workload (default: the 576k-atom mixed fit; fit_fp64: the "
                         "116k-atom FP64 fit alone, with its legs)")
    ap.add_argument("--cpu-sample-cfgs", type=int, default=48,
                    help="fit_fp64 headline: configurations of the oracle sample")
    ap.add_argument("--cpu-full", action="store_true",
                    help="time the FP64 oracle on the whole 116k-atom fit (about 30 GB of host "
                         "memory, minutes of CPU time) instead of a sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--refine-steps", type=int, default=3,
                    help="most FP64 refinement steps of a mixed fit")
    ap.add_argument("--refine-tol", type=float, default=1e-14,
                    help="the 576k-atom fit stops refining once the error left in c is "
                         "predicted below this (relative)")
    ap.add_argument("--no-virial", action="store_true",
                    help="skip timing the virial, two-body, variance and CUR legs")
    ap.add_argument("--no-predict", action="store_true",
                    help="skip the predict / backward leg on the 65,536-atom predict workload")
    ap.add_argument("--no-fp64-legs", action="store_true",
                    help="default headline: skip the 116k-atom legs after the large fit")
    ap.add_argument("--stream-blocks", type=int, default=4,
                    help="configuration groups of the streamed-fit leg (0: skip it)")
    ap.add_argument("--large-rows", type=int, default=435000,
                    help="observation rows per batch of the 576k-atom fit (at most ~515k: "
                         "the QR panel holds a batch's rows across the grid)")
    ap.add_argument("--knm-only", action="store_true",
                    help="576k-atom workload: time only the K_NM assembly of every batch "
                         "(Jacobians drawn, BF16X3 rows built), no fold, solve or refinement")
    ap.add_argument("--predict-only", action="store_true",
                    help="time only the predict / backward leg on the 65,536-atom predict "
                         "workload and print its figures")
    ap.add_argument("--large-cfgs", type=int, default=0,
                    help="576k-atom fit: fit only its first N configurations (0: all 4000)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build runs the GAP hot path on one GPU only; "
              "--gpus must be 1 (multi-GPU sharding is described, not built).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    import paper_2310_03921_amd as gapx

    if args.workload == "fit_fp64":
        peaks = measured_peaks(torch)
        out = fit_fp64_legs(args, torch, synth, gapx, headline=True)
        out["measured_peaks"] = peaks
        if peaks:
            rf = out["roofline"]
            rf["peak_measured"] = peaks["fp64_tflops"]
            rf["frac_of_measured_peak"] = rf["achieved"] / peaks["fp64_tflops"]
            rf["peak_measured_random_operands"] = peaks["fp64_random_operands_tflops"]
            rf["frac_of_measured_random_operand_peak"] = (
                rf["achieved"] / peaks["fp64_random_operands_tflops"])
        print(json.dumps(out), flush=True)
        return
    if args.knm_only:
        print(json.dumps(large_knm_bench(args, torch, synth, gapx)), flush=True)
        return
    if args.predict_only:
        gap = gapx.Gap(0)
        out = {"leg": "predict_workload", "steps": args.steps,
               **predict_leg(args, torch, synth, gapx, gap)}
        gap.close()
        print(json.dumps(out), flush=True)
        return
    peaks = measured_peaks(torch)
    line = large_fit_bench(args, torch, synth, gapx)
    line["measured_peaks"] = peaks
    if peaks:
        rf = line["roofline"]
        rf["peak_measured"] = peaks["bf16_tflops"] / 3.0
        rf["frac_of_measured_peak"] = rf["achieved"] / rf["peak_measured"]
        rf["peak_measured_random_operands"] = peaks["bf16_random_operands_tflops"] / 3.0
        rf["frac_of_measured_random_operand_peak"] = (
            rf["achieved"] / rf["peak_measured_random_operands"])
    if not args.no_cpu_baseline:
        log("timing the FP64 CPU oracle on a sample of the large fit")
        line["cpu_baseline"] = cpu_baseline_large(synth)
    if not args.no_fp64_legs:
        line["fit_fp64_116k"] = fit_fp64_legs(args, torch, synth, gapx, headline=False)
    print(json.dumps(line), flush=True)


def predict_leg(args, torch, synth, gapx, gap):
    """Predict and backward on the predict workload (65,536 atoms, D = 1000,
    M = 4000, FP32 descriptors and Jacobians): energies + descriptor gradients
    (two GEMM-shaped contractions), the force contraction over the Jacobians
    (an HBM stream), and the backward (three contractions), FP64 and BF16X3."""
    wp = synth.WORKLOADS["predict"]
    log(f"generating {wp.name} on the host")
    bp = synth.generate(wp)
    Xp = synth.sparse_points(wp, bp)
    atp = gapx.Atoms.from_host(bp.cfg_ptr, bp.desc, bp.pair_ptr, bp.pair_j, bp.jac,
                               desc_dtype=torch.float32, jac_dtype=torch.float32)
    bp.jac = None
    spp = gapx.Sparse.from_host(Xp, wp.zeta, wp.delta)
    cp = torch.tensor(synth.predict_coefficients(wp), device="cuda")
    ge = torch.ones(atp.n_atoms, dtype=torch.float64, device="cuda")
    torch.cuda.synchronize()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        tt = []
        for _ in range(args.steps):
            ts = time.perf_counter()
            out_ = fn()
            torch.cuda.synchronize()
            tt.append(time.perf_counter() - ts)
        return float(np.mean(tt)), out_
    Np, Mp, Dp = atp.n_atoms, wp.M, wp.D
    fwd_flops = 2.0 * 2.0 * Np * Mp * Dp
    bwd_flops = 3.0 * 2.0 * Np * Mp * Dp
    jbytes = float(atp.n_pairs) * 3 * Dp * 4
    pred = {"workload": describe(wp, bp), "energy_and_gradient_s": {}, "backward_s": {},
            "energy_and_gradient_tflops": {}, "backward_tflops": {}}
    dEdd = None
    for prec in ("fp64", "bf16x3"):
        t_f, o = timed(lambda: gap.predict(atp, spp, cp, prec, e_atom=True, e_cfg=True,
                                           dEdd=True, forces=False))
        t_b, _ = timed(lambda: gap.predict_backward(atp, spp, cp, ge, prec))
        pred["energy_and_gradient_s"][prec] = t_f
        pred["backward_s"][prec] = t_b
        pred["energy_and_gradient_tflops"][prec] = fwd_flops / t_f / 1e12
        pred["backward_tflops"][prec] = bwd_flops / t_b / 1e12
        if prec == "fp64":
            dEdd = o["dEdd"]
    t_j, _ = timed(lambda: gap.forces(atp, dEdd))
    pred["forces_from_gradients_s"] = t_j
    pred["forces_jacobian_bytes"] = jbytes
    pred["forces_hbm_tbs"] = jbytes / t_j / 1e12
    log(f"predict workload: energies + gradients {pred['energy_and_gradient_s']['fp64'] * 1e3:.1f} ms "
        f"FP64 / {pred['energy_and_gradient_s']['bf16x3'] * 1e3:.1f} ms BF16X3, forces "
        f"{t_j * 1e3:.1f} ms ({pred['forces_hbm_tbs']:.2f} TB/s of Jacobians), backward "
        f"{pred['backward_s']['fp64'] * 1e3:.1f} / {pred['backward_s']['bf16x3'] * 1e3:.1f} ms")
    del atp, dEdd
    return pred


def fit_fp64_legs(args, torch, synth, gapx, headline):
    """The 116k-atom FP64 fit and its legs (mixed, streamed, variance, CUR, two-body,
    virial rows, the predict workload); with headline, the CPU oracle too."""
    w = synth.WORKLOADS["fit_fp64"]
    log(f"generating {w.name} on the host")
    t0 = time.perf_counter()
    b = synth.generate(w)
    X = synth.sparse_points(w, b)
    log(f"generated {b.n_atoms} atoms / {b.n_pairs} pairs in {time.perf_counter() - t0:.1f} s")

    torch.cuda.set_device(0)
    gap = gapx.Gap(0)
    atoms = gapx.Atoms.from_host(b.cfg_ptr, b.desc, b.pair_ptr, b.pair_j, b.jac)
    sp = gapx.Sparse.from_host(X, w.zeta, w.delta)
    n_rows, M, D = b.n_rows, w.M, w.D
    # targets from the hidden coefficients (GPU predict) plus seeded noise
    cstar = torch.tensor(synth.hidden_coefficients(w), device="cuda")
    pr = gap.predict(atoms, sp, cstar, e_atom=False, e_cfg=True, forces=True)
    y = torch.cat([pr["e_cfg"], pr["forces"].reshape(-1)])
    y += torch.tensor(synth.noise(w, b.cfg_ids, b.counts), device="cuda")
    sigma = torch.tensor(synth.sigma_rows(w, b.counts), device="cuda")
    A = gap.design_buffer(atoms, sp)
    Kmm = gapx.colmajor(M, M, M)
    torch.cuda.synchronize()
    log(f"inputs resident: J {atoms.jac.numel() * atoms.jac.element_size() / 1e9:.1f} GB, "
        f"A {A.numel() * 8 / 1e9:.1f} GB")

    def step():
        gap.build_kmm(sp, out=Kmm)
        gap.build_knm(atoms, sp, out=A)
        return gap.fit(A, n_rows, Kmm, y, sigma, w.jitter, sp)

    for i in range(args.warmup):
        step()
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")
    gap.timing(True)
    gap.timing_read(reset=True)
    torch.cuda.synchronize()
    times = []
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        c, info = step()
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        log(f"step {i + 1}/{args.steps}: {times[-1] * 1e3:.1f} ms")
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    stages = gap.timing_read(reset=True)
    gap.timing(False)
    per = {k: (v[0] / args.steps) for k, v in stages.items() if v[1] > 0}

    fit_s = total / args.steps
    knm_ms = per.get("pair_transpose", 0) + per.get("energy_rows", 0) + per.get("force_rows", 0)
    knm_flops = 2.0 * M * D * (b.n_atoms + 3.0 * b.n_pairs)
    force_flops = 2.0 * 3.0 * b.n_pairs * M * D
    force_ms = per.get("force_rows", float("nan"))
    achieved = force_flops / (force_ms * 1e-3) / 1e12
    qr_flops = 2.0 * (n_rows + M) * (M + 1) ** 2 - 2.0 / 3.0 * (M + 1) ** 3
    qr_ms = per.get("qr_panel", 0) + per.get("qr_update", 0)

    assert torch.isfinite(c).all().item(), "non-finite coefficients"
    c64 = c.clone()

    mixed = None
    if not args.no_mixed:
        def mixed_step():
            gap.build_kmm(sp, out=Kmm)
            gap.build_knm(atoms, sp, precision="bf16x3", out=A)
            return gap.fit(A, n_rows, Kmm, y, sigma, w.jitter, sp, train=atoms,
                           refine_steps=args.refine_steps)
        # the untimed first fit reports |A^T r| after its last step as well; the
        # timed fits skip that diagnostic residual pass (c is the same)
        _, minfo = mixed_step()
        torch.cuda.synchronize()
        log("mixed warmup done")
        gap.set_fit_report(False)
        gap.timing(True)
        gap.timing_read(reset=True)
        tm = []
        for i in range(args.steps):
            ts = time.perf_counter()
            cmx, tinfo = mixed_step()
            torch.cuda.synchronize()
            tm.append(time.perf_counter() - ts)
            log(f"mixed step {i + 1}/{args.steps}: {tm[-1] * 1e3:.1f} ms")
        mst = gap.timing_read(reset=True)
        gap.timing(False)
        gap.set_fit_report(True)
        assert tinfo["refine_done"] == minfo["refine_done"]
        mper = {k: (v[0] / args.steps) for k, v in mst.items() if v[1] > 0}
        # accuracy against the FP64 fit and against the noise-free truth (forces from c*)
        ref = gap.predict(atoms, sp, cstar, e_atom=False, e_cfg=True, forces=True)
        p64 = gap.predict(atoms, sp, c64, e_atom=False, e_cfg=True, forces=True)
        pmx = gap.predict(atoms, sp, cmx, e_atom=False, e_cfg=True, forces=True)
        nat = torch.tensor(b.counts, dtype=torch.float64, device="cuda")

        def rmse(a, b_):
            return float(torch.sqrt(torch.mean((a - b_) ** 2)))
        mknm = mper.get("split_bf16", 0) + mper.get("pair_transpose", 0) + \
            mper.get("energy_rows", 0) + mper.get("force_rows", 0)
        mforce_flops_exec = 3.0 * 2.0 * 3.0 * b.n_pairs * M * (((D + 31) // 32) * 32)
        mixed = {
            "fit_s": float(np.mean(tm)),
            "refine_steps": args.refine_steps,
            "refine_done": minfo["refine_done"],
            "timed_fit_final_residual": False,
            "stage_ms": {k: round(v, 3) for k, v in mper.items()},
            "knm_ms": mknm,
            "knm_gflops_algorithmic": knm_flops / (mknm * 1e-3) / 1e9 if mknm > 0 else None,
            "force_rows_bf16_tflops_executed": mforce_flops_exec / (mper.get("force_rows", float("nan")) * 1e-3) / 1e12,
            "force_rows_bf16_frac_of_2500": mforce_flops_exec / (mper.get("force_rows", float("nan")) * 1e-3) / 1e12 / 2500.0,
            "c_rel_vs_fp64": float(torch.linalg.norm(cmx - c64) / torch.linalg.norm(c64)),
            "resid_norm": minfo["resid_norm"],
            "force_rmse_vs_truth": {"fp64": rmse(p64["forces"], ref["forces"]),
                                    "mixed": rmse(pmx["forces"], ref["forces"])},
            "force_rmse_mixed_vs_fp64": rmse(pmx["forces"], p64["forces"]),
            "energy_rmse_per_atom_vs_truth": {
                "fp64": rmse(p64["e_cfg"] / nat, ref["e_cfg"] / nat),
                "mixed": rmse(pmx["e_cfg"] / nat, ref["e_cfg"] / nat)},
        }
        log(f"mixed fit {mixed['fit_s'] * 1e3:.1f} ms, c rel vs fp64 {mixed['c_rel_vs_fp64']:.2e}")

    streamed = None
    if args.stream_blocks > 0:
        # The same fit with A never held whole: K_NM rows of each group of
        # configurations are built into the block area of the fold state and
        # folded into the triangular factor of [A | b].
        bounds = np.linspace(0, b.n_cfg, args.stream_blocks + 1).round().astype(int)
        parts = []
        for c0, c1 in zip(bounds[:-1], bounds[1:]):
            c0, c1 = int(c0), int(c1)
            sub = atoms.configs(c0, c1)
            a0, a1 = int(b.cfg_ptr[c0]), int(b.cfg_ptr[c1])
            rows = torch.cat([torch.arange(c0, c1), b.n_cfg + torch.arange(3 * a0, 3 * a1)]).cuda()
            parts.append((sub, y[rows].contiguous(), sigma[rows].contiguous()))
        T = gap.fold_buffer(M, max(p[0].n_rows for p in parts))

        def stream_step():
            gap.build_kmm(sp, out=Kmm)
            gap.fold_init(T, M, Kmm, w.jitter)
            for sub, yb, sb in parts:
                gap.build_knm_block(sub, sp, T)
                gap.fold_rows(T, M, sub.n_rows, yb, sb)
            return gap.fold_solve(T, M)
        stream_step()
        torch.cuda.synchronize()
        log("streamed warmup done")
        gap.timing(True)
        gap.timing_read(reset=True)
        ts_ = []
        for i in range(args.steps):
            ts = time.perf_counter()
            cst, lres, _ = stream_step()
            torch.cuda.synchronize()
            ts_.append(time.perf_counter() - ts)
            log(f"streamed step {i + 1}/{args.steps}: {ts_[-1] * 1e3:.1f} ms")
        sst = gap.timing_read(reset=True)
        gap.timing(False)
        streamed = {
            "fit_s": float(np.mean(ts_)),
            "blocks": len(parts),
            "rows_per_block_max": max(p[0].n_rows for p in parts),
            "state_bytes": T.numel() * 8,
            "design_bytes_one_shot": A.numel() * 8,
            "stage_ms": {k: round(v[0] / args.steps, 3) for k, v in sst.items() if v[1] > 0},
            "c_rel_vs_one_shot": float(torch.linalg.norm(cst - c64) / torch.linalg.norm(c64)),
            "lsq_resid_norm": lres,
        }
        log(f"streamed fit {streamed['fit_s'] * 1e3:.1f} ms in {len(parts)} blocks, "
            f"state {streamed['state_bytes'] / 1e9:.2f} GB vs A {streamed['design_bytes_one_shot'] / 1e9:.2f} GB, "
            f"c rel vs one-shot {streamed['c_rel_vs_one_shot']:.2e}")

    variance = None
    if not args.no_virial:
        # predictive variance of every atom's local energy from the FP64 fit's R
        # (A holds the last fit's factor unless the mixed leg refitted it)
        A64 = gap.design_buffer(atoms, sp)
        gap.build_kmm(sp, out=Kmm)
        gap.build_knm(atoms, sp, out=A64)
        gap.fit(A64, n_rows, Kmm, y, sigma, w.jitter, sp)
        gap.predict_variance(atoms, sp, Kmm, w.jitter, A64)
        torch.cuda.synchronize()
        tvv = []
        for i in range(args.steps):
            ts = time.perf_counter()
            vv = gap.predict_variance(atoms, sp, Kmm, w.jitter, A64)
            torch.cuda.synchronize()
            tvv.append(time.perf_counter() - ts)
        variance = {"atoms": b.n_atoms, "call_s": float(np.mean(tvv)),
                    "min": float(vv.min()), "max": float(vv.max())}
        log(f"predictive variance of {b.n_atoms} atoms: {variance['call_s'] * 1e3:.1f} ms")
        del A64, vv

    cur = None
    if not args.no_virial:
        # CUR selection of M sparse points among all the atoms' descriptors
        gap.select_cur(atoms, M, 0.0)
        torch.cuda.synchronize()
        tc = []
        for i in range(args.steps):
            ts = time.perf_counter()
            gap.select_cur(atoms, M, 0.0)
            tc.append(time.perf_counter() - ts)
        cur = {"atoms": b.n_atoms, "n_sparse": M, "call_s": float(np.mean(tc))}
        log(f"CUR selection of {M} of {b.n_atoms} atoms: {cur['call_s'] * 1e3:.1f} ms")

    twobody = None
    virial = None
    if not args.no_virial:
        # nine virial rows per configuration, same pairs and Jacobians
        pr_ = torch.tensor(synth.pair_vectors(w, b), device="cuda")
        # a 32-point two-body SE block over the same pairs (every observation row)
        k2 = gapx.SE2b.from_host(synth.sparse_distances(w, 32))
        K2 = gap.build_2b_rows(atoms, k2, pr_)
        torch.cuda.synchronize()
        t2 = []
        for i in range(args.steps):
            ts = time.perf_counter()
            gap.build_2b_rows(atoms, k2, pr_, out=K2)
            gap.sync()
            t2.append(time.perf_counter() - ts)
        twobody = {"rows": n_rows, "M": 32, "pairs": b.n_pairs, "call_s": float(np.mean(t2))}
        log(f"two-body rows ({n_rows} x 32): {twobody['call_s'] * 1e3:.1f} ms")
        del K2
        Kv = gapx.colmajor(9 * b.n_cfg, M)
        gap.build_virial_rows(atoms, sp, pr_, out=Kv)
        torch.cuda.synchronize()
        gap.timing(True)
        gap.timing_read(reset=True)
        tv = []
        for i in range(args.steps):
            ts = time.perf_counter()
            gap.build_virial_rows(atoms, sp, pr_, out=Kv)
            gap.sync()
            tv.append(time.perf_counter() - ts)
        vst = gap.timing_read(reset=True)
        gap.timing(False)
        vk = vst["force_rows"][0] / args.steps
        virial = {"rows": 9 * b.n_cfg, "call_s": float(np.mean(tv)),
                  "kernel_ms": vk, "kernel_tflops": force_flops / (vk * 1e-3) / 1e12,
                  "stage_ms": {k: round(v[0] / args.steps, 3) for k, v in vst.items() if v[1] > 0}}
        log(f"virial rows ({9 * b.n_cfg}): call {virial['call_s'] * 1e3:.1f} ms, kernel {vk:.1f} ms "
            f"({virial['kernel_tflops']:.1f} TFLOP/s)")
        del Kv, pr_

    pred = None
    if not args.no_predict:
        del A
        torch.cuda.empty_cache()
        pred = predict_leg(args, torch, synth, gapx, gap)

    cpu = None
    if headline and not args.no_cpu_baseline:
        log("timing the FP64 CPU oracle" + (" on the whole fit" if args.cpu_full else " on a sample"))
        cpu = cpu_baseline_full(w, b, X) if args.cpu_full else cpu_baseline(w, b, X, args.cpu_sample_cfgs)

    out = {
        "metric": METRIC,
        "value": fit_s,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": fit_s * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": describe(w, b), "precision": "fp64",
                   "n_rows": n_rows, "M": M, "D": D},
        "knm_gflops": knm_flops / (knm_ms * 1e-3) / 1e9 if knm_ms > 0 else None,
        "knm_ms": knm_ms,
        "qr_ms": qr_ms,
        "qr_tflops": qr_flops / (qr_ms * 1e-3) / 1e12 if qr_ms > 0 else None,
        "stage_ms": {k: round(v, 3) for k, v in per.items()},
        "roofline": {"kernel": "k_force_rows (force observation rows, FP64 MFMA)",
                     "bound": "mfma", "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS,
                     "traffic": force_traffic_bytes(w), "traffic_unit": "bytes per launch",
                     "flops_per_launch": force_flops},
        "cpu_baseline": cpu,
        "mixed_bf16x3": mixed,
        "streamed_fp64": streamed,
        "virial_rows_fp64": virial,
        "two_body_rows_fp64": twobody,
        "predict_workload": pred,
        "predict_variance_fp64": variance,
        "cur_selection": cur,
        "fit_info": {"min_abs_rdiag": info["min_abs_rdiag"], "max_abs_rdiag": info["max_abs_rdiag"]},
    }
    return out


if __name__ == "__main__":
    main()
