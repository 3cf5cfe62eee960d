"""Wegner-dual transverse-field Ising oracle for 2+1D lattices (test infrastructure only).

In two space dimensions the Z2 gauge theory is dual to the transverse-field
Ising model (Sec. 3.2, the duality H(g) = g H~(1/g) with H~ the Ising model).
With one Ising spin tau on every plaquette p:

    U_p          <->  tau^x_p
    sigma^x_l    <->  tau^z_p tau^z_p'     (p, p' = the two plaquettes sharing l)
    G_i          <->  1

and the gauge-invariant sector with every 't Hooft loop V_mu = +1 maps onto
the even sector (prod_p tau^x_p = +1) of the Ising model on the dual torus.
Each Trotter factor maps onto its dual exactly:

    exp(+i a sum_l sigma^x_l)   <->  exp(+i a sum_l tau^z_p tau^z_p')   (diagonal)
    exp(+i t sum_p U_p)         <->  prod_p exp(+i t tau^x_p)

and |+>^{N_l} (every sigma^x_l = +1, no electric loop) maps onto
(|0...0> + |1...1>)/sqrt 2.  A 2^{N_l}-amplitude evolution therefore has an
exact 2^{N_p}-amplitude image, e.g. 2^16 amplitudes for the 32-link 4x4
torus.  Plain numpy, FP64.
"""
from __future__ import annotations

import numpy as np


class DualIsing:
    def __init__(self, plaq: np.ndarray, n_links: int):
        """plaq: the gauge lattice's plaquette link lists (n_p x 4)."""
        plaq = np.asarray(plaq)
        self.n = plaq.shape[0]
        owners = [[] for _ in range(n_links)]
        for p, links in enumerate(plaq):
            for l in links:
                owners[int(l)].append(p)
        if any(len(o) != 2 for o in owners):
            raise ValueError("duality needs every link on exactly two plaquettes (d = 2)")
        self.bonds = np.array(owners, dtype=np.int64)  # bond l joins plaquettes bonds[l]
        b = np.arange(1 << self.n, dtype=np.int64)
        zz = np.zeros(1 << self.n, dtype=np.int64)
        for p, q in self.bonds:
            same = ((b >> p) & 1) == ((b >> q) & 1)
            zz += np.where(same, 1, -1)
        self.zz = zz  # sum_l tau^z_p tau^z_p' on each basis state

    def ghz(self) -> np.ndarray:
        psi = np.zeros(1 << self.n, dtype=np.complex128)
        psi[0] = psi[-1] = 1 / np.sqrt(2)
        return psi

    def _rx_all(self, psi: np.ndarray, t: float) -> np.ndarray:
        """prod_p exp(+i t tau^x_p)."""
        c, s = np.cos(t), np.sin(t)
        for p in range(self.n):
            v = psi.reshape(-1, 2, 1 << p)
            a0 = v[:, 0, :].copy()
            a1 = v[:, 1, :].copy()
            v[:, 0, :] = c * a0 + 1j * s * a1
            v[:, 1, :] = 1j * s * a0 + c * a1
        return psi

    def evolve(self, psi, dt, cx, cz, order: int) -> np.ndarray:
        """Image of the gauge-theory Trotter product (eq. (a) / eq. (s))."""
        for a, b in zip(cx, cz):
            if order == 1:
                psi *= np.exp(1j * dt * a * self.zz)
                self._rx_all(psi, dt * b)
            else:
                self._rx_all(psi, 0.5 * dt * b)
                psi *= np.exp(1j * dt * a * self.zz)
                self._rx_all(psi, 0.5 * dt * b)
        return psi

    # observables: images of <U_p>, <sigma^x_l>, Wegner-Wilson loops
    def expect_tx(self, psi, plaquettes) -> float:
        """<prod_{p in set} tau^x_p>: the image of a contractible Wilson loop enclosing the set."""
        flip = 0
        for p in plaquettes:
            flip |= 1 << int(p)
        idx = np.arange(1 << self.n) ^ flip
        return float(np.real(np.vdot(psi, psi[idx])) / np.vdot(psi, psi).real)

    def expect_bond(self, psi, l: int) -> float:
        p, q = self.bonds[l]
        b = np.arange(1 << self.n)
        sign = np.where(((b >> p) & 1) == ((b >> q) & 1), 1.0, -1.0)
        return float(np.sum(sign * np.abs(psi) ** 2) / np.vdot(psi, psi).real)

    def hamiltonian(self, J: float, h: float) -> np.ndarray:
        """Dense -J sum_bonds tau^z tau^z - h sum_p tau^x (small n only)."""
        dim = 1 << self.n
        H = np.diag(-J * self.zz.astype(np.complex128))
        for p in range(self.n):
            idx = np.arange(dim)
            H[idx ^ (1 << p), idx] += -h
        return H

    def even_projector(self) -> np.ndarray:
        dim = 1 << self.n
        idx = np.arange(dim)
        P = 0.5 * np.eye(dim, dtype=np.complex128)
        P[idx ^ (dim - 1), idx] += 0.5
        return P
