"""QAOA statevector on a cone, its <Z_u Z_v>, and a forward-mode gradient (O4, O5, O7).

Sec. 2.2 defines the state
    |beta, gamma>_p = U_B(beta_p) U_P(gamma_p) ... U_B(beta_1) U_P(gamma_1) |+>^k
with U_P(gamma) = exp(-i gamma H) and U_B(beta) = prod_j exp(-i beta X_j).
For MaxCut (Sec. 2.4) H = 1/2 sum_(a,b) w_ab (I - Z_a Z_b) is diagonal: its value on
|x> is the weighted cut C(x) = sum_(a,b) w_ab [x_a != x_b].  So U_P multiplies the
amplitude of |x> by exp(-i gamma C(x)).

Basis index convention: bit j of the integer x is the value of qubit j.

The gradient is propagated forward (one tangent state per parameter), which is a
different algorithm from the adjoint sweep of the GPU path:
    d/dgamma_l of U_P(gamma_l) = -i C U_P(gamma_l),
    d/dbeta_l  of U_B(beta_l)  = -i (sum_j X_j) U_B(beta_l),
    d<O>/dtheta = 2 Re <psi| O |dpsi/dtheta>.
"""
from __future__ import annotations

import numpy as np


def cut_values(k: int, edges, weights=None) -> np.ndarray:
    """C(x) for every basis state x of k qubits (float64 [2^k])."""
    x = np.arange(1 << k, dtype=np.int64)
    c = np.zeros(1 << k, dtype=np.float64)
    if weights is None:
        weights = np.ones(len(edges))
    for (a, b), wab in zip(edges, weights):
        c += float(wab) * (((x >> a) ^ (x >> b)) & 1)
    return c


def _apply_x_rotation(psi: np.ndarray, k: int, j: int, beta: float) -> np.ndarray:
    """exp(-i beta X_j) on qubit j."""
    s = psi.reshape(1 << (k - 1 - j), 2, 1 << j)
    a0, a1 = s[:, 0, :], s[:, 1, :]
    c, sn = np.cos(beta), np.sin(beta)
    out = np.empty_like(s)
    out[:, 0, :] = c * a0 - 1j * sn * a1
    out[:, 1, :] = c * a1 - 1j * sn * a0
    return out.reshape(-1)


def apply_mixer(psi: np.ndarray, k: int, beta: float) -> np.ndarray:
    """U_B(beta) = prod_j exp(-i beta X_j) on all k qubits."""
    for j in range(k):
        psi = _apply_x_rotation(psi, k, j, beta)
    return psi


def apply_x(psi: np.ndarray, k: int, j: int) -> np.ndarray:
    """Pauli X on qubit j (bit flip of bit j)."""
    return psi.reshape(1 << (k - 1 - j), 2, 1 << j)[:, ::-1, :].reshape(-1)


def apply_b(psi: np.ndarray, k: int) -> np.ndarray:
    """B = sum_j X_j."""
    out = np.zeros_like(psi)
    for j in range(k):
        out += apply_x(psi, k, j)
    return out


def qaoa_state(k: int, cut: np.ndarray, gammas, betas) -> np.ndarray:
    """The depth-p QAOA state on k qubits (complex128 [2^k])."""
    psi = np.full(1 << k, 2.0 ** (-k / 2), dtype=np.complex128)
    for g, b in zip(gammas, betas):
        psi = psi * np.exp(-1j * g * cut)
        psi = apply_mixer(psi, k, b)
    return psi


def zz_sign(k: int, a: int = 0, b: int = 1) -> np.ndarray:
    x = np.arange(1 << k, dtype=np.int64)
    return 1.0 - 2.0 * (((x >> a) ^ (x >> b)) & 1)


def zz_expectation(psi: np.ndarray, k: int, a: int = 0, b: int = 1) -> float:
    """<psi| Z_a Z_b |psi>."""
    return float(np.sum(np.abs(psi) ** 2 * zz_sign(k, a, b)))


def zz_and_grad(k: int, cut: np.ndarray, gammas, betas):
    """Return (zz, dzz/dgamma [p], dzz/dbeta [p]) for the observable Z_0 Z_1."""
    p = len(gammas)
    psi = np.full(1 << k, 2.0 ** (-k / 2), dtype=np.complex128)
    tang = np.zeros((2 * p, 1 << k), dtype=np.complex128)   # [gamma_1..p, beta_1..p]
    for l in range(p):
        ph = np.exp(-1j * gammas[l] * cut)
        psi = ph * psi
        tang = tang * ph[None, :]
        tang[l] += -1j * cut * psi
        psi = apply_mixer(psi, k, betas[l])
        for t in range(2 * p):
            tang[t] = apply_mixer(tang[t], k, betas[l])
        tang[p + l] += -1j * apply_b(psi, k)
    sgn = zz_sign(k)
    zz = float(np.sum(np.abs(psi) ** 2 * sgn))
    d = 2.0 * np.real(np.conj(psi * sgn)[None, :] * tang).sum(axis=1)
    return zz, d[:p].copy(), d[p:].copy()
