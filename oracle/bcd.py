"""Sequential block coordinate descent (BCD) and DBCD.  TEST INFRASTRUCTURE ONLY.

``naive_bcd_*`` is the textbook sequential BCD that DID reorganises (Section 4.1): every
coordinate is minimised with its closed form evaluated *from scratch*, with no carried
residual and no W/V messages:

* c_ij := [ b_i^T (x_j - sum_{k != i} b_k c_kj) / (b_i^T b_i) ]_+   (eq. sol:c_ij, first line)
  for i = 1..K within each column j, every column j;
* b_i  := [ sum_j (x_j - B c_j + b_i c_ij) c_ij / sum_j c_ij^2 ]_+ (eq. sol:b_i 2)
  for i = 1..K, after the whole C half.

The experiments section states that DID takes exactly the iterations of BCD and DBCD
(paragraph "Correctness"); the tests use this module to pin the oracle's DID to that
claim.  It is written with explicit Python loops on purpose and is meant for tiny inputs.

``dbcd_iteration`` is Alg. 2 (DBCD): the same C half, then for every i one reduction of
(y_j, z_j) = ((e_j + b_i c_ij) c_ij, c_ij^2) over all columns and b_i := [y/z]_+.
"""

from __future__ import annotations

import numpy as np


def _pos(z):
    return z if z > 0.0 else 0.0


def naive_bcd_iteration(X, B, C):
    """One sequential BCD iteration on float64 arrays, in place on B and C."""
    M, N = X.shape
    K = B.shape[1]
    for j in range(N):
        for i in range(K):
            nb = float(B[:, i] @ B[:, i])
            if not nb > 0.0:
                continue
            a = X[:, j].copy()
            for k in range(K):
                if k != i:
                    a -= B[:, k] * C[k, j]
            C[i, j] = _pos(float(B[:, i] @ a) / nb)
    for i in range(K):
        z = float(C[i, :] @ C[i, :])
        if not z > 0.0:
            continue
        A = X.copy()
        for k in range(K):
            if k != i:
                A -= np.outer(B[:, k], C[k, :])
        y = A @ C[i, :]
        for m in range(M):
            B[m, i] = _pos(float(y[m]) / z)


def naive_bcd_run(X, B0, C0, T, eps=None):
    """T naive BCD iterations; with ``eps`` stop once ||E^t||^2 <= eps ||E^0||^2.

    Returns (B, C, f, t_stop) with f[t] = 1/2 ||X - B^t C^t||^2 and t_stop the stopping
    iteration (T if the rule never fired).
    """
    X = np.asarray(X, np.float64)
    B = np.array(B0, dtype=np.float64, copy=True)
    C = np.array(C0, dtype=np.float64, copy=True)

    def fval():
        E = X - B @ C
        return 0.5 * float(np.sum(E * E))

    f = [fval()]
    for t in range(1, T + 1):
        naive_bcd_iteration(X, B, C)
        f.append(fval())
        if eps is not None and f[-1] <= eps * f[0]:
            return B, C, np.array(f), t
    return B, C, np.array(f), T


def dbcd_iteration(X, B, C, blocks):
    """One DBCD iteration (Alg. 2) on float64 arrays, in place on B and C.

    C half as in Alg. 2 (e_j := x_j - B c_j, then eq. up:c for i = 1..K).  B half: for each
    i, every block forms sum_j y_j and sum_j z_j over its columns, the partials are added
    in block order (one reduction per i), and b_i := [y/z]_+; then e_j is updated by
    e_j := e_j - b_i c_ij after having added back the old b_i c_ij.
    """
    M, N = X.shape
    K = B.shape[1]
    E = X - B @ C
    for i in range(K):
        nb = float(B[:, i] @ B[:, i])
        if not nb > 0.0:
            continue
        E += np.outer(B[:, i], C[i, :])
        c_new = np.where((B[:, i] @ E) / nb > 0.0, (B[:, i] @ E) / nb, 0.0)
        C[i, :] = c_new
        E -= np.outer(B[:, i], C[i, :])
    for i in range(K):
        E += np.outer(B[:, i], C[i, :])
        y = np.zeros(M)
        z = 0.0
        for a, b in blocks:
            y += E[:, a:b] @ C[i, a:b]
            z += float(C[i, a:b] @ C[i, a:b])
        if z > 0.0:
            B[:, i] = np.where(y / z > 0.0, y / z, 0.0)
        E -= np.outer(B[:, i], C[i, :])
    return E
