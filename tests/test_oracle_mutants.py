"""Plant plausible mistakes in the oracle (on the CPU) and check that the pins catch them.

Each mutant replaces one step of ``oracle.did`` for the duration of a test.  The pins used
are the exact worked example with clipping (golden file) and DID == sequential BCD; a
mutant that survived both would mean the pins are too weak to trust the oracle.
"""

import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import bcd
from oracle import did as D

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "worked_examples.json")


def _mat(rows):
    return np.array([[float(Fraction(v)) for v in r] for r in rows])


def _pins_hold():
    with open(GOLDEN) as fh:
        g = json.load(fh)["k2_clipping"]
    X, B0, C0 = _mat(g["X"]), _mat(g["B0"]), _mat(g["C0"])
    B, C, f = D.did_run(X, B0, C0, 1)
    ok_golden = (np.allclose(B, _mat(g["B1"]), atol=1e-12) and np.allclose(C, _mat(g["C1"]), atol=1e-12)
                 and abs(f[1] - float(Fraction(g["f1"]))) < 1e-12)
    rng = np.random.default_rng(99)
    X = rng.random((6, 8)) * 3
    B0, C0 = rng.random((6, 3)), rng.random((3, 8))
    B, C, f = D.did_run(X, B0, C0, 5, P=2)
    Bn, Cn, fn, _ = bcd.naive_bcd_run(X, B0, C0, 5)
    ok_bcd = np.allclose(B, Bn, atol=1e-10) and np.allclose(C, Cn, atol=1e-10)
    return ok_golden and ok_bcd


def _b_half_no_cross_term(B, W, V):
    M, K = B.shape
    dB = np.zeros((M, K))
    for i in range(K):
        if V[i, i] > 0:
            b_new = D.project(B[:, i] + W[:, i] / V[i, i])
            dB[:, i] = b_new - B[:, i]
            B[:, i] = b_new
    return dB


def _b_half_transposed_v(B, W, V):
    M, K = B.shape
    dB = np.zeros((M, K))
    Vf = V + np.tril(V, -1).T
    for i in range(K):
        if V[i, i] > 0:
            corr = dB[:, i + 1:] @ (Vf[i, i + 1:] / V[i, i])  # wrong index range
            b_new = D.project(B[:, i] + W[:, i] / V[i, i] - corr)
            dB[:, i] = b_new - B[:, i]
            B[:, i] = b_new
    return dB


def _c_half_wrong_sign(B, C, E):
    K = B.shape[1]
    n = np.einsum("mk,mk->k", B, B)
    for i in range(K):
        if n[i] > 0:
            c_new = D.project(C[i, :] + (B[:, i] @ E) / n[i])
            E += np.outer(B[:, i], c_new - C[i, :])  # sign flipped
            C[i, :] = c_new
    return n


def _c_half_stale_residual(B, C, E):
    K = B.shape[1]
    n = np.einsum("mk,mk->k", B, B)
    E0 = E.copy()
    for i in range(K):
        if n[i] > 0:
            c_new = D.project(C[i, :] + (B[:, i] @ E0) / n[i])  # residual never refreshed
            E -= np.outer(B[:, i], c_new - C[i, :])
            C[i, :] = c_new
    return n


_messages = D.messages


def _messages_w_transposed_blocks(E, C, blocks):
    W, V = _messages(E, C, blocks)
    return W, V.T.copy()  # upper instead of lower triangle: v_ik read as zero for k < i


@pytest.mark.parametrize("target,mutant", [
    ("b_half", _b_half_no_cross_term),
    ("b_half", _b_half_transposed_v),
    ("c_half", _c_half_wrong_sign),
    ("c_half", _c_half_stale_residual),
    ("messages", _messages_w_transposed_blocks),
])
def test_pins_catch_planted_mistake(monkeypatch, target, mutant):
    assert _pins_hold()
    monkeypatch.setattr(D, target, mutant)
    assert not _pins_hold()
