"""Seeded synthetic workloads for the GAP regression hot path.

This module only draws random numbers and lays them out; it holds none of the
method's arithmetic (no kernel, no covariance, no solve).  Both the GPU library
tests and the FP64 CPU oracle consume what it produces.

The paper's training databases (Si, HEA, SiC, QM9-GW; Sec. "Application
examples") are not used.  Stand-ins follow the structure the method consumes
(Sec. "Representations" and "Regression"): per-atom descriptor vectors, the
descriptor Jacobian for each (atom, neighbour slot) pair, and a configuration
-> atoms map (the operator L-hat of eq. GP_L).

Recipe (stated once, applied per configuration so that any configuration can be
regenerated alone, which is what sampled parity checks at full size rely on):

* atom counts n_c ~ U{lo..hi}                    stream [seed, 0]
* per configuration c, stream [seed, 1, c]:
    descriptors d_i ~ N(0, I_D), divided by their 2-norm in FP64, then cast
    to the workload's descriptor dtype;
    neighbour slots j(i, k) ~ U{0..n_c-1} with replacement (the atom itself
    may appear; duplicates add, read as periodic images);
    Jacobian slots J[i, k, alpha, :] ~ N(0, 0.1^2) drawn in the Jacobian dtype.
* sparse set: M distinct atom indices, uniform without replacement,
  stream [seed, 2]; x_m is a bit copy of the chosen descriptor.
* hidden coefficients c* ~ N(0, 1), stream [seed, 3].
* observation noise, stream [seed, 4, c]: energy ~ N(0, sigma_E^2 * n_c),
  forces ~ N(0, sigma_F^2) per component.
* pair displacement vectors (virial and two-body rows), stream [seed, 5, c]:
  uniform in a ball of radius 5.
* sparse distances of the two-body descriptor, stream [seed, 6]: uniform in
  [0.5, 5].
* device-drawn Jacobians (workloads whose Jacobians do not fit in device
  memory; ``device_jacobians``): element e = (p * 3 + alpha) * D + d of the
  global pair p is 0.1 * N(0, 1) from the counter-based stream (seed, JAC_TAG)
  of ``normal_gen.hip`` (Philox4x32-10 + Box-Muller), so a batch of
  configurations, or any single one, is regenerated alone on the device and
  copied back for the oracle when a check needs its values.
"""
from __future__ import annotations

import ctypes
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, replace

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    n_cfg: int
    atoms_lo: int
    atoms_hi: int
    D: int
    nb: int
    M: int
    zeta: int = 4
    delta: float = 1.0
    sigma_e: float = 1e-3      # per-atom energy regularisation (variance scaled by n_c)
    sigma_f: float = 1e-2      # per force component
    jitter: float = 1e-8
    desc_dtype: str = "f64"
    jac_dtype: str = "f64"
    precision: str = "fp64"    # contraction precision of the GPU path: fp64 | bf16x3

    def with_(self, **kw) -> "Workload":
        return replace(self, **kw)


# Workloads with the shapes of the paper's fits (D from compressed SOAP, zeta=4,
# sigma and jitter values of the Si example table).
WORKLOADS = {
    "fit_small": Workload("fit_small", 1, 50, 8, 64, 252, 20, 200),
    "fit_fp64": Workload("fit_fp64", 2, 1000, 16, 216, 252, 30, 2000),
    "fit_small_mixed": Workload("fit_small_mixed", 1, 50, 8, 64, 252, 20, 200,
                                precision="bf16x3"),
    "predict": Workload("predict", 4, 256, 256, 256, 1000, 40, 4000,
                        desc_dtype="f32", jac_dtype="f32"),
    "fit_large_mixed": Workload("fit_large_mixed", 5, 4000, 32, 256, 1500, 40, 8000,
                                desc_dtype="f32", jac_dtype="f32", precision="bf16x3"),
}

_NP = {"f64": np.float64, "f32": np.float32}


@dataclass
class Batch:
    """A generated batch of configurations, host arrays.

    desc    [N_at, D]          row-major descriptors
    cfg_ptr [n_cfg + 1] int64  atoms of configuration c are cfg_ptr[c]:cfg_ptr[c+1]
    pair_ptr[N_at + 1] int64   source-major CSR of (atom, slot) pairs
    pair_j  [n_pairs]  int32   global index of the atom the slot points at
    jac     [n_pairs, 3, D]    d(desc_i)/d(r_{j(i,k), alpha}) for pair (i, k)
    """
    w: Workload
    cfg_ids: np.ndarray
    counts: np.ndarray
    cfg_ptr: np.ndarray
    desc: np.ndarray
    pair_ptr: np.ndarray
    pair_j: np.ndarray
    jac: np.ndarray | None

    @property
    def n_atoms(self) -> int:
        return int(self.cfg_ptr[-1])

    @property
    def n_cfg(self) -> int:
        return len(self.cfg_ptr) - 1

    @property
    def n_pairs(self) -> int:
        return int(self.pair_ptr[-1])

    @property
    def n_rows(self) -> int:
        return self.n_cfg + 3 * self.n_atoms


def atom_counts(w: Workload) -> np.ndarray:
    rng = np.random.default_rng([w.seed, 0])
    return rng.integers(w.atoms_lo, w.atoms_hi + 1, size=w.n_cfg).astype(np.int64)


def _draw_config(w: Workload, c: int, n: int, jac: bool, desc_out, jac_out, nbr_out):
    rng = np.random.default_rng([w.seed, 1, c])
    d = rng.standard_normal((n, w.D))
    d /= np.sqrt(np.einsum("ij,ij->i", d, d))[:, None]
    desc_out[...] = d.astype(_NP[w.desc_dtype])
    nbr_out[...] = rng.integers(0, n, size=(n, w.nb))
    if jac:
        jdt = _NP[w.jac_dtype]
        rng.standard_normal(out=jac_out.reshape(-1), dtype=jdt)
        jac_out *= jdt(0.1)


def generate(w: Workload, cfg_ids=None, jac: bool = True, threads: int | None = None) -> Batch:
    """Generate the configurations ``cfg_ids`` (default: all) of workload ``w``.

    Atom and pair indices in the returned batch are local to the returned
    configurations (renumbered from zero), so a sampled subset is itself a
    valid batch.
    """
    counts_all = atom_counts(w)
    cfg_ids = np.arange(w.n_cfg) if cfg_ids is None else np.asarray(cfg_ids, dtype=np.int64)
    counts = counts_all[cfg_ids]
    cfg_ptr = np.zeros(len(cfg_ids) + 1, dtype=np.int64)
    np.cumsum(counts, out=cfg_ptr[1:])
    n_at = int(cfg_ptr[-1])
    desc = np.empty((n_at, w.D), dtype=_NP[w.desc_dtype])
    nbr = np.empty((n_at, w.nb), dtype=np.int64)
    jac_arr = np.empty((n_at * w.nb, 3, w.D), dtype=_NP[w.jac_dtype]) if jac else None

    def work(t):
        c, lo, hi = int(cfg_ids[t]), int(cfg_ptr[t]), int(cfg_ptr[t + 1])
        _draw_config(w, c, hi - lo, jac, desc[lo:hi], None if not jac else
                     jac_arr[lo * w.nb:hi * w.nb].reshape(hi - lo, w.nb, 3, w.D), nbr[lo:hi])
        nbr[lo:hi] += lo

    nthreads = threads or min(16, os.cpu_count() or 1)
    if nthreads > 1 and len(cfg_ids) > 1:
        with ThreadPoolExecutor(nthreads) as ex:
            list(ex.map(work, range(len(cfg_ids))))
    else:
        for t in range(len(cfg_ids)):
            work(t)
    pair_ptr = np.arange(n_at + 1, dtype=np.int64) * w.nb
    return Batch(w, cfg_ids, counts, cfg_ptr, desc, pair_ptr,
                 nbr.reshape(-1).astype(np.int32), jac_arr)


def global_atom_offsets(w: Workload) -> np.ndarray:
    """cfg_ptr of the full workload (global atom numbering)."""
    ptr = np.zeros(w.n_cfg + 1, dtype=np.int64)
    np.cumsum(atom_counts(w), out=ptr[1:])
    return ptr


def sparse_indices(w: Workload) -> np.ndarray:
    """M distinct global atom indices, uniform without replacement."""
    n_at = int(global_atom_offsets(w)[-1])
    if w.M > n_at:
        raise ValueError("more sparse points than atoms")
    return np.random.default_rng([w.seed, 2]).choice(n_at, size=w.M, replace=False)


def sparse_points(w: Workload, batch: Batch | None = None) -> np.ndarray:
    """X [M, D] FP64: bit copies of the selected training descriptors.

    With ``batch`` covering all configurations the rows are copied from it;
    otherwise only the configurations holding sparse atoms are regenerated.
    """
    idx = sparse_indices(w)
    if batch is not None and len(batch.cfg_ids) == w.n_cfg:
        return batch.desc[idx].astype(np.float64)
    gptr = global_atom_offsets(w)
    cfg_of = np.searchsorted(gptr, idx, side="right") - 1
    X = np.empty((w.M, w.D), dtype=np.float64)

    def work(c):
        n = int(gptr[c + 1] - gptr[c])
        d = np.empty((n, w.D), dtype=_NP[w.desc_dtype])
        nbr = np.empty((n, w.nb), dtype=np.int64)
        _draw_config(w, int(c), n, False, d, None, nbr)
        sel = np.nonzero(cfg_of == c)[0]
        X[sel] = d[idx[sel] - gptr[c]].astype(np.float64)

    cfgs = np.unique(cfg_of)
    nthreads = min(16, os.cpu_count() or 1)
    if nthreads > 1 and len(cfgs) > 1:
        with ThreadPoolExecutor(nthreads) as ex:
            list(ex.map(work, cfgs))
    else:
        for c in cfgs:
            work(c)
    return X


def hidden_coefficients(w: Workload) -> np.ndarray:
    return np.random.default_rng([w.seed, 3]).standard_normal(w.M)


def sigma_rows(w: Workload, counts: np.ndarray) -> np.ndarray:
    """Per-observation sigma: energies sigma_E*sqrt(n_c), then 3 per atom sigma_F."""
    n_at = int(np.sum(counts))
    return np.concatenate([w.sigma_e * np.sqrt(counts.astype(np.float64)),
                           np.full(3 * n_at, w.sigma_f)])


def noise(w: Workload, cfg_ids: np.ndarray, counts: np.ndarray) -> np.ndarray:
    """Observation noise in row order (energies of the batch, then forces)."""
    e = np.empty(len(cfg_ids))
    f = []
    for t, (c, n) in enumerate(zip(cfg_ids, counts)):
        rng = np.random.default_rng([w.seed, 4, int(c)])
        e[t] = rng.normal(0.0, w.sigma_e * np.sqrt(float(n)))
        f.append(rng.normal(0.0, w.sigma_f, size=3 * int(n)))
    return np.concatenate([e] + f)


def pair_vectors(w: Workload, batch: Batch, r_cut: float = 5.0) -> np.ndarray:
    """Displacement r_j - r_i of every pair (i, k), FP64 [n_pairs, 3].

    Stream [seed, 5, c] per configuration: directions uniform on the sphere,
    lengths r_cut * U^(1/3) (uniform in the cutoff ball).  A stand-in for the
    periodic-image vectors of a real neighbour list; only virial rows use it.
    """
    out = np.empty((batch.n_pairs, 3))
    for t, c in enumerate(batch.cfg_ids):
        a0, a1 = int(batch.cfg_ptr[t]), int(batch.cfg_ptr[t + 1])
        p0, p1 = int(batch.pair_ptr[a0]), int(batch.pair_ptr[a1])
        rng = np.random.default_rng([w.seed, 5, int(c)])
        v = rng.standard_normal((p1 - p0, 3))
        v /= np.maximum(np.linalg.norm(v, axis=1, keepdims=True), 1e-300)
        out[p0:p1] = v * (r_cut * rng.random((p1 - p0, 1)) ** (1.0 / 3.0))
    return out


def sparse_distances(w: Workload, M: int, lo: float = 0.5, hi: float = 5.0) -> np.ndarray:
    """Sparse points of a two-body distance descriptor: M distances uniform in
    [lo, hi], sorted, stream [seed, 6]."""
    return np.sort(np.random.default_rng([w.seed, 6]).uniform(lo, hi, size=M))


def predict_coefficients(w: Workload) -> np.ndarray:
    """Coefficients for a predict-only workload, c ~ N(0, 1)."""
    return hidden_coefficients(w)


# ------------------------------------------------------------------------
# Counter-based generator (Philox4x32-10; Salmon et al., SC'11): the host
# definition, and the device library that draws the same stream on the GPU.

JAC_TAG = 0x4A414331          # key word 1 of the device-drawn Jacobian stream
_PHILOX_M = (0xD2511F53, 0xCD9E8D57)
_PHILOX_W = (0x9E3779B9, 0xBB67AE85)
_LIBSYNTH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libsynth.so")
_synth_lib = None


def philox4x32_10(counters: np.ndarray, key0: int, key1: int) -> np.ndarray:
    """Philox4x32-10 of uint32 counters [n, 4] under key (key0, key1): ten
    rounds of the published round function, the key bumped by the Weyl
    constants between rounds.  Returns uint32 [n, 4]."""
    c = [np.asarray(counters, dtype=np.uint64)[:, i].copy() for i in range(4)]
    mask = np.uint64(0xFFFFFFFF)
    k0, k1 = np.uint64(key0 & 0xFFFFFFFF), np.uint64(key1 & 0xFFFFFFFF)
    for _ in range(10):
        p0 = np.uint64(_PHILOX_M[0]) * c[0]
        p1 = np.uint64(_PHILOX_M[1]) * c[2]
        c = [((p1 >> np.uint64(32)) ^ c[1] ^ k0) & mask, p1 & mask,
             ((p0 >> np.uint64(32)) ^ c[3] ^ k1) & mask, p0 & mask]
        k0 = (k0 + np.uint64(_PHILOX_W[0])) & mask
        k1 = (k1 + np.uint64(_PHILOX_W[1])) & mask
    return np.stack(c, axis=1).astype(np.uint32)


def stream_words(seed: int, tag: int, g0: int, n_groups: int) -> np.ndarray:
    """Host words of groups g0 .. g0 + n_groups - 1 of stream (seed, tag): counter
    (g mod 2^32, g / 2^32, 0, 0), key (seed mod 2^32, tag)."""
    g = np.arange(g0, g0 + n_groups, dtype=np.uint64)
    ctr = np.zeros((n_groups, 4), dtype=np.uint64)
    ctr[:, 0] = g & np.uint64(0xFFFFFFFF)
    ctr[:, 1] = g >> np.uint64(32)
    return philox4x32_10(ctr, seed, tag)


def box_muller(words: np.ndarray) -> np.ndarray:
    """The four normals of each group of words, in FP64 (host reference of the
    device transform, which works in FP32)."""
    w = np.asarray(words, dtype=np.float64)
    out = np.empty_like(w)
    for a, b in ((0, 1), (2, 3)):
        u = (w[:, a] + 1.0) * 2.0 ** -32
        v = w[:, b] * 2.0 ** -32
        r = np.sqrt(-2.0 * np.log(u))
        out[:, a] = r * np.cos(2.0 * np.pi * v)
        out[:, b] = r * np.sin(2.0 * np.pi * v)
    return out


def synth_lib():
    """The device generator library (built by synth/build.py)."""
    global _synth_lib
    if _synth_lib is None:
        if not os.path.exists(_LIBSYNTH):
            raise ImportError(f"{_LIBSYNTH} is missing: run synth.build.build()")
        L = ctypes.CDLL(_LIBSYNTH)
        L.synth_philox_words.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p]
        L.synth_philox_words.restype = ctypes.c_int
        L.synth_normal_rows_f32.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                            ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                            ctypes.c_int64, ctypes.c_float, ctypes.c_void_p]
        L.synth_normal_rows_f32.restype = ctypes.c_int
        _synth_lib = L
    return _synth_lib


def _stream_ptr(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def device_words(seed: int, tag: int, g0: int, n_groups: int, device="cuda"):
    """Device words of groups g0 .. g0 + n_groups - 1 (uint32 as int32 tensor [n, 4])."""
    import torch
    out = torch.empty(max(n_groups, 1), 4, dtype=torch.int32, device=device)
    st = synth_lib().synth_philox_words(_stream_ptr(out), seed & 0xFFFFFFFF, tag, g0, n_groups,
                                        ctypes.c_void_p(out.data_ptr()))
    if st != 0:
        raise RuntimeError(f"synth_philox_words failed ({st})")
    return out[:n_groups]


def device_normal_rows(out, seed: int, tag: int, e0: int, D: int, scale: float):
    """Fill the FP32 device tensor out [rows, ld] (ld >= D) with scale * N(0, 1)
    elements e0 + r D + d of stream (seed, tag); padding columns untouched."""
    rows, ld = out.shape[0], out.shape[-1]
    st = synth_lib().synth_normal_rows_f32(_stream_ptr(out), seed, tag, e0, rows, D, ld,
                                           float(scale), ctypes.c_void_p(out.data_ptr()))
    if st != 0:
        raise RuntimeError(f"synth_normal_rows_f32 failed ({st})")
    return out


def jacobian_ld(D: int) -> int:
    """Row length of the device-drawn Jacobians: D rounded up to 32 FP32 values."""
    return (D + 31) // 32 * 32


def device_jacobians(w: Workload, cfg0: int, cfg1: int, out=None, device="cuda"):
    """Jacobian slots of configurations [cfg0, cfg1) drawn on the device, FP32
    [n_pairs, 3, ld] (ld = D rounded up to 32, so that every row starts on a
    128-byte line; padding zero when ``out`` is new).
    Pair p of the whole workload (global numbering) holds elements
    (p * 3 + alpha) * D + d of stream (seed, JAC_TAG), times 0.1."""
    import torch
    gptr = global_atom_offsets(w)
    p0, p1 = int(gptr[cfg0]) * w.nb, int(gptr[cfg1]) * w.nb
    ld = jacobian_ld(w.D)
    if out is None:
        out = torch.zeros(p1 - p0, 3, ld, dtype=torch.float32, device=device)
    elif out.shape[0] < p1 - p0 or out.shape[1] != 3 or out.shape[2] < w.D or \
            out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous FP32 tensor [>= n_pairs, 3, >= D]")
    device_normal_rows(out.view(-1, out.shape[2])[:3 * (p1 - p0)], w.seed, JAC_TAG,
                       p0 * 3 * w.D, w.D, 0.1)
    return out[:p1 - p0]
