"""DID in plain NumPy FP64: the oracle.  TEST INFRASTRUCTURE ONLY (see package docstring).

Every function follows the paper (Gao & Chu, "DID: Distributed Incremental Block
Coordinate Descent for Nonnegative Matrix Factorization", AAAI-18, arXiv 1802.08938)
in its order and notation:

* problem: minimise f(B, C) = 1/2 ||X - BC||_F^2 over B, C >= 0, with X (M x N) whose
  columns are samples, B (M x K) the basis and C (K x N) the coordinates
  (Introduction, eq. opt:nmf);
* X and C are split into P column blocks X_p, C_p; B is replicated (Section
  "Distributed ADMM", the column-separable objective, reused by Section 4);
* one DID iteration (Section 4, Alg. 3):
    1. e_j := x_j - B c_j for every column j,
    2. for i = 1..K: c_ij updated by eq. up:c (the closed form of eq. sol:c_ij applied
       against the running residual e_j),
    3. messages W_j = [e_j c_1j ... e_j c_Kj] and V_j = tril(c_j c_j^T) (eqs. W_j, V_j),
       summed over all columns (the single Allreduce; here a sum over blocks p in
       ascending order),
    4. for i = 1..K: b_i := [b_i + w_i/v_ii - sum_{k<i} (v_ik/v_ii) delta b_k]_+ and
       delta b_i := b_i^{t+1} - b_i^t (Section "Incremental Update for b_i").

Readings taken where the paper is silent:

* the residual is carried across iterations and updated explicitly by
  E := E - delta b_i c_i^r (Section "Incremental Update for b_i"); Alg. 3 recomputes
  e_j at the start of every iteration, which is equal in exact arithmetic.  The
  carried residual is checked against a fresh X - BC by ``did_run(check=True)``;
* the c-update uses the single-line form of eq. sol:c_ij (c + b^T e / b^T b, then
  project) with e updated by b_i (c_new - c_old), algebraically equal to eq. up:c;
* a zero denominator (b_i^T b_i = 0 or v_ii = 0, the failure mode the experiments
  section warns about) skips that coordinate: its value and delta stay unchanged/zero;
* [z]_+ = max{0, z} returns +0.0 for every z <= 0.

The C half is written vectorised over columns j (columns are independent, Section 4.1),
with the K coordinates taken in ascending order; this is the same arithmetic as a loop
over j.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "project",
    "objective",
    "residual",
    "column_blocks",
    "c_half",
    "messages",
    "b_half",
    "did_iteration",
    "did_run",
    "iterations_to_tolerance",
]


def project(z):
    """[z]_+ = max{0, z} elementwise (closed forms of HALS, Section 2), +0.0 for z <= 0."""
    z = np.asarray(z, dtype=np.float64)
    return np.where(z > 0.0, z, 0.0)


def residual(X, B, C):
    """E = X - BC (Section 4, 'E = X - BC, the most current residual matrix')."""
    return np.asarray(X, np.float64) - np.asarray(B, np.float64) @ np.asarray(C, np.float64)


def objective(X, B, C):
    """f(B, C) = 1/2 ||X - BC||_F^2 (eq. opt:nmf)."""
    E = residual(X, B, C)
    return 0.5 * float(np.sum(E * E))


def column_blocks(N, P):
    """Contiguous column blocks [(a_p, b_p)] with sum N_p = N (column partition of X and C).

    The first N mod P blocks get one extra column.  P is clipped to [1, N].
    """
    P = max(1, min(int(P), int(N)))
    base, extra = divmod(int(N), P)
    out, a = [], 0
    for p in range(P):
        n = base + (1 if p < extra else 0)
        out.append((a, a + n))
        a += n
    return out


def c_half(B, C, E):
    """Coordinate sweep over the rows of C (Alg. 3, 'Update C'), in place on C and E.

    For each i = 1..K in ascending order and every column j (independent):
        c_ij := [c_ij + b_i^T e_j / (b_i^T b_i)]_+          (eq. sol:c_ij)
        e_j  := e_j - b_i (c_ij^new - c_ij^old)              (eq. up:c, first+third lines)
    B is fixed during the half, so b_i^T b_i is taken once.
    Returns the vector of norms n_i = b_i^T b_i that was used.
    """
    K = B.shape[1]
    n = np.einsum("mk,mk->k", B, B)
    for i in range(K):
        if not n[i] > 0.0:  # zero column of B: the closed form is undefined; skip
            continue
        g = B[:, i] @ E  # b_i^T e_j for all j
        c_new = project(C[i, :] + g / n[i])
        E -= np.outer(B[:, i], c_new - C[i, :])
        C[i, :] = c_new
    return n


def messages(E, C, blocks):
    """Messages of Alg. 3 summed over the blocks (eqs. W_j, V_j; the one Allreduce).

    W = sum_j W_j = E C^T (M x K), V = sum_j V_j = tril(C C^T) (K x K), each block's
    partial formed from its own columns and the partials added in ascending block order.
    """
    M, K = E.shape[0], C.shape[0]
    W = np.zeros((M, K))
    V = np.zeros((K, K))
    for a, b in blocks:
        Ep, Cp = E[:, a:b], C[:, a:b]
        W += Ep @ Cp.T
        V += np.tril(Cp @ Cp.T)
    return W, V


def b_half(B, W, V):
    """Incremental update of the columns of B (Alg. 3, 'Update B'), in place on B.

    For i = 1..K:
        b_i^{t+1} := [b_i^t + w_i/v_ii - sum_{k<i} (v_ik/v_ii) delta b_k]_+
        delta b_i := b_i^{t+1} - b_i^t
    Returns delta B (M x K).
    """
    M, K = B.shape
    dB = np.zeros((M, K))
    for i in range(K):
        vii = V[i, i]
        if not vii > 0.0:  # zero row of C: skip, delta b_i = 0
            continue
        corr = dB[:, :i] @ (V[i, :i] / vii)
        b_new = project(B[:, i] + W[:, i] / vii - corr)
        dB[:, i] = b_new - B[:, i]
        B[:, i] = b_new
    return dB


def did_iteration(X, B, C, E, blocks):
    """One DID iteration (Alg. 3) on float64 arrays, in place on B, C and E.

    E enters as X - BC for the current (B, C) and leaves as X - B^{t+1} C^{t+1}, carried by
    E := E - delta b_i c_i^r (Section 'Incremental Update for b_i').
    Returns (W, V, dB) for inspection.
    """
    c_half(B, C, E)
    W, V = messages(E, C, blocks)
    dB = b_half(B, W, V)
    E -= dB @ C
    return W, V, dB


def did_run(X, B0, C0, T, P=1, check=False, tol_R=1e-10, history=True):
    """Run T DID iterations from (B0, C0).

    Returns (B, C, f) where f[t] = f(B^t, C^t) for t = 0..T (f[0] at the initial point,
    f[t] after the full iteration t).  With ``check=True`` every iteration asserts the
    invariants the method guarantees: B, C >= 0, the carried residual equals a fresh
    X - BC to ``tol_R * max(1, max X)``, and f does not increase (after the C half and
    after the whole iteration, up to 1e-12 relative rounding slack).
    """
    X = np.asarray(X, np.float64)
    B = np.array(B0, dtype=np.float64, copy=True)
    C = np.array(C0, dtype=np.float64, copy=True)
    M, N = X.shape
    blocks = column_blocks(N, P)
    E = residual(X, B, C)
    f = [0.5 * float(np.sum(E * E))]
    scale = max(1.0, float(np.max(X)) if X.size else 1.0)
    for _ in range(T):
        if check:
            c_half(B, C, E)
            fc = 0.5 * float(np.sum(E * E))
            assert fc <= f[-1] * (1 + 1e-12) + 1e-300, "objective rose in the C half"
            assert np.max(np.abs(E - residual(X, B, C)), initial=0.0) <= tol_R * scale
            W, V = messages(E, C, blocks)
            dB = b_half(B, W, V)
            E -= dB @ C
        else:
            did_iteration(X, B, C, E, blocks)
        ft = 0.5 * float(np.sum(E * E))
        if check:
            assert np.all(B >= 0.0) and np.all(C >= 0.0)
            assert np.max(np.abs(E - residual(X, B, C)), initial=0.0) <= tol_R * scale
            assert ft <= fc * (1 + 1e-12) + 1e-300, "objective rose in the B half"
        if history:
            f.append(ft)
    return B, C, np.array(f)


def iterations_to_tolerance(X, B0, C0, eps=1e-6, max_iter=1000, P=1):
    """Iterations until ||E^t||_F^2 <= eps ||E^0||_F^2 (the experiments' stopping rule).

    Returns (t, f) with t the first iteration meeting the rule (or max_iter if none did)
    and f the objective history up to it.
    """
    X = np.asarray(X, np.float64)
    B = np.array(B0, dtype=np.float64, copy=True)
    C = np.array(C0, dtype=np.float64, copy=True)
    blocks = column_blocks(X.shape[1], P)
    E = residual(X, B, C)
    e0 = float(np.sum(E * E))
    f = [0.5 * e0]
    for t in range(1, max_iter + 1):
        did_iteration(X, B, C, E, blocks)
        et = float(np.sum(E * E))
        f.append(0.5 * et)
        if et <= eps * e0:
            return t, np.array(f)
    return max_iter, np.array(f)
