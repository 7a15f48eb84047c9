"""Structural Jacobian pattern, brute-force symbolic fill, no-pivot LU (oracle; tests only).

The paper's Processes declare at initialization which Jacobian elements they touch, so the
solver can use a sparse Jacobian (Table of Process functions, get_used_jacobian_elements),
and the linear solver is a sparse direct LU (Sect. 2.4.1, KLU). Here:

* ``structural_pattern``: (i, j) is used when species j is a reactant of some expanded
  reaction in which species i takes part (as reactant or product), or j is one of the
  species a reaction's Parameter is diagnosed from (Sect. 2.2.2); the diagonal is always
  included (the Newton matrix is I - gamma J).
* ``symbolic_fill``: plain boolean Gaussian elimination in a given pivot order: eliminating
  pivot k makes (i, j) nonzero for every i after k with (i, k) nonzero and every j after k
  with (k, j) nonzero.
* ``lu_nopivot``: dense Doolittle LU in the given order without pivoting (the device LU
  uses a static order and no pivoting).
"""
import numpy as np


def structural_pattern(x):
    n = x.n_state
    P = np.eye(n, dtype=bool)
    for xr in x.rxns:
        members = set(xr.react) | set(xr.prod)
        for j in set(xr.react) | set(xr.param_species or []) | set(xr.radius_species or []):
            for i in members:
                P[i, j] = True
    return P


def symbolic_fill(P, order):
    """Filled pattern, in the permuted index space (row/col t is original order[t])."""
    A = P[np.ix_(order, order)].copy()
    n = A.shape[0]
    for k in range(n):
        rows = [i for i in range(k + 1, n) if A[i, k]]
        cols = [j for j in range(k + 1, n) if A[k, j]]
        for i in rows:
            for j in cols:
                A[i, j] = True
    return A


def lu_nopivot(M):
    """In-place-style Doolittle LU without pivoting: returns the combined L\\U matrix."""
    A = np.array(M, dtype=np.float64, copy=True)
    n = A.shape[0]
    for k in range(n):
        for i in range(k + 1, n):
            if A[i, k] != 0.0:
                A[i, k] /= A[k, k]
                A[i, k + 1:] -= A[i, k] * A[k, k + 1:]
    return A


def lu_solve_nopivot(LU, b):
    n = LU.shape[0]
    x = np.array(b, dtype=np.float64, copy=True)
    for i in range(n):
        x[i] -= LU[i, :i] @ x[:i]
    for i in range(n - 1, -1, -1):
        x[i] = (x[i] - LU[i, i + 1:] @ x[i + 1:]) / LU[i, i]
    return x
