"""Pins of the topological-sector experiment (Sec. 3.5) on the oracle: Wegner-Wilson lines
move the projected Z ground state between the sectors of the 't Hooft operators, the
sectors are conserved by the evolution, and each sector's adiabatic energy respects the
variational bound of its exact ground energy."""
import numpy as np
import pytest

import oracle
from oracle import ed


def _apply_z(psi, links):
    b = np.arange(len(psi), dtype=np.int64)
    par = np.zeros_like(b)
    for q in links:
        par ^= (b >> int(q)) & 1
    return np.where(par == 1, -psi, psi)


def test_wilson_lines_flip_the_thooft_sectors():
    """W along mu shares one link with V_mu (anticommutes) and none with V_nu, nu != mu."""
    for d, L in [(2, (2, 3)), (2, (3, 3)), (3, (2, 2, 2))]:
        lat = oracle.Lattice(d, L)
        for mu in range(d):
            for nu in range(d):
                shared = set(lat.line(0, mu).tolist()) & set(lat.thooft(nu))
                assert len(shared) == (1 if mu == nu else 0)
    lat = oracle.Lattice(2, (2, 3))
    psi0 = oracle.zground_state(lat)
    for mu in range(2):
        psi = _apply_z(psi0, lat.line(0, mu))
        for nu in range(2):
            v = oracle.expect_x(psi, lat.N, lat.thooft(nu))
            assert abs(v - (-1.0 if mu == nu else 1.0)) < 1e-12


def _sector_projector(lat, signs):
    N = lat.N
    P = ed.sector_projector(N, lat.stars, [])
    for mu, s in enumerate(signs):
        V = ed.pauli_product(N, lat.thooft(mu), ed.SX)
        P = P @ (0.5 * (np.eye(1 << N) + s * V))
    return P


@pytest.mark.parametrize("signs", [(1, 1), (-1, 1), (-1, -1)])
def test_sector_energies_respect_their_ground_energies(signs):
    lat = oracle.Lattice(2, (2, 2))
    psi = oracle.zground_state(lat)
    for mu, s in enumerate(signs):
        if s < 0:
            psi = _apply_z(psi, lat.line(0, mu))
    rows = oracle.adiabatic_scan(lat, psi, 1.0, 10, 20, 1.0, 2, loops=[])
    P = _sector_projector(lat, signs)
    for g, _, z, x, n2 in rows:
        e0 = ed.sector_spectrum(ed.hamiltonian(lat.N, lat.plaq, g, 1.0), P)[0]
        h = z + g * x
        assert h >= e0 - 1e-9
        assert h - e0 < 0.05
