"""Dense exact-diagonalisation references for tiny lattices (test infrastructure only).

Operators are built as Kronecker products of 2x2 Pauli matrices, which is an
independent construction from the amplitude loops in ``lgt_oracle.c``: with
bit q of the basis index being link q, an operator P on link q is
``kron(I_{2^(N-1-q)}, P, I_{2^q})``.

The Hamiltonian is H = -cx sum_l sigma^x_l - cz sum_p U_p (Sec. 2.1 with
g = cx / cz when cz = 1), and exp(-i t H) is taken from ``scipy.linalg.expm``.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

I2 = np.eye(2, dtype=np.complex128)
SX = np.array([[0, 1], [1, 0]], dtype=np.complex128)
SZ = np.array([[1, 0], [0, -1]], dtype=np.complex128)


def op_on(N: int, q: int, P: np.ndarray) -> np.ndarray:
    return np.kron(np.kron(np.eye(1 << (N - 1 - q)), P), np.eye(1 << q))


def pauli_product(N: int, links, P: np.ndarray) -> np.ndarray:
    M = np.eye(1 << N, dtype=np.complex128)
    for q in links:
        M = M @ op_on(N, int(q), P)
    return M


def h_links(N: int) -> np.ndarray:
    """sum_l sigma^x_l"""
    return sum(op_on(N, q, SX) for q in range(N))


def h_plaq(N: int, plaq) -> np.ndarray:
    """sum_p U_p with U_p = prod_{l in p} sigma^z_l"""
    return sum(pauli_product(N, p, SZ) for p in plaq)


def hamiltonian(N: int, plaq, cx: float, cz: float) -> np.ndarray:
    return -cx * h_links(N) - cz * h_plaq(N, plaq)


def trotter_step_matrix(N, plaq, dt, cx, cz, order: int) -> np.ndarray:
    """eq. (a): e^{-i dt Hz} e^{-i dt Hx};  eq. (s): e^{-i dt Hz/2} e^{-i dt Hx} e^{-i dt Hz/2}."""
    Ux = sla.expm(1j * dt * cx * h_links(N))
    Uz_full = sla.expm(1j * dt * cz * h_plaq(N, plaq))
    if order == 1:
        return Uz_full @ Ux
    Uz_half = sla.expm(0.5j * dt * cz * h_plaq(N, plaq))
    return Uz_half @ Ux @ Uz_half


def exact_stepwise(psi0: np.ndarray, N, plaq, dt, cx, cz) -> np.ndarray:
    """prod_j exp(-i dt H_j) psi0: the stepwise Hamiltonian of Sec. 2.2, no splitting."""
    psi = psi0.copy()
    Hx = h_links(N)
    Hz = h_plaq(N, plaq)
    for a, b in zip(cx, cz):
        w, V = np.linalg.eigh(-a * Hx - b * Hz)
        psi = V @ (np.exp(-1j * dt * w) * (V.conj().T @ psi))
    return psi


def sector_projector(N: int, stars, tHooft) -> np.ndarray:
    """Projector onto G_i = +1 for every star and V_mu = +1 for the given 't Hooft loops."""
    P = np.eye(1 << N, dtype=np.complex128)
    for links in list(stars) + list(tHooft):
        G = pauli_product(N, links, SX)
        P = P @ (0.5 * (np.eye(1 << N) + G))
    return P


def sector_spectrum(H: np.ndarray, P: np.ndarray) -> np.ndarray:
    """Eigenvalues of H restricted to range(P) (P an orthogonal projector commuting with H)."""
    w, V = np.linalg.eigh(P)
    B = V[:, w > 0.5]
    return np.linalg.eigvalsh(B.conj().T @ H @ B)
