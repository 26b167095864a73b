"""The oracle reproduces the hand-worked example in tests/golden/hand_example.json."""
import json
import os

import numpy as np

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))


def load_hand_example():
    with open(os.path.join(HERE, "golden", "hand_example.json")) as f:
        g = json.load(f)
    for k in ("X", "desc", "jac", "Kmm", "Knm", "c", "e_atom", "e_cfg", "dEdd", "forces"):
        g[k] = np.array(g[k], dtype=np.float64)
    for k in ("cfg_ptr", "pair_ptr"):
        g[k] = np.array(g[k], dtype=np.int64)
    g["pair_j"] = np.array(g["pair_j"], dtype=np.int32)
    return g


def test_hand_example_covariances():
    g = load_hand_example()
    assert np.allclose(oracle.build_kmm(g["X"], g["zeta"], g["delta"]), g["Kmm"], rtol=1e-14, atol=1e-14)
    K = oracle.build_knm(g["cfg_ptr"], g["desc"], g["pair_ptr"], g["pair_j"], g["jac"], g["X"],
                         g["zeta"], g["delta"])
    assert np.allclose(K, g["Knm"], rtol=1e-14, atol=1e-14)


def test_hand_example_predict():
    g = load_hand_example()
    e, ec, dd, F = oracle.predict(g["cfg_ptr"], g["desc"], g["pair_ptr"], g["pair_j"], g["jac"],
                                  g["X"], g["c"], g["zeta"], g["delta"])
    assert np.allclose(e, g["e_atom"], rtol=1e-14, atol=1e-14)
    assert np.allclose(ec, g["e_cfg"], rtol=1e-14, atol=1e-14)
    assert np.allclose(dd, g["dEdd"], rtol=1e-14, atol=1e-14)
    assert np.allclose(F, g["forces"], rtol=1e-14, atol=1e-14)
