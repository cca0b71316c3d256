"""Dense brute force on tiny tori (test infrastructure).

The walk operator U = sum_h T_h (x) U_h (Sec. 2) written out as an explicit
(sV x sV) matrix. Index of (component c, site n) is c*V + lin(n) with lin the
row-major site index. U^t is then taken by repeated squaring and, separately,
by eigen-decomposition.
"""
import numpy as np


def dense_walk(table, N, d):
    s = next(iter(table.values())).shape[0]
    V = N ** d
    sites = np.stack(np.meshgrid(*([np.arange(N)] * d), indexing="ij"), axis=-1).reshape(-1, d)
    lin = np.ravel_multi_index(sites.T, (N,) * d)
    M = np.zeros((s * V, s * V), dtype=np.complex128)
    for off, U in table.items():
        src = np.ravel_multi_index(((sites + np.array(off)) % N).T, (N,) * d)
        for i in range(s):
            for j in range(s):
                if U[i, j] != 0:
                    M[i * V + lin, j * V + src] += U[i, j]
    return M


def power_matpow(M, t):
    if t >= 0:
        return np.linalg.matrix_power(M, t)
    return np.linalg.matrix_power(M.conj().T, -t)


def power_eig(M, t):
    w, Vec = np.linalg.eig(M)
    return (Vec * (w ** t)) @ np.linalg.inv(Vec)


def apply_dense(Mt, psi):
    s = psi.shape[0]
    return (Mt @ psi.reshape(-1)).reshape(psi.shape)
