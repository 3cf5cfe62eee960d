"""Pins of the oracle's stepwise adiabatic scan (Sec. 2.2, Sec. 3): an independent
dual-Ising image, the pure-Z limit and the variational bound with the exact ground state."""
import numpy as np
import pytest

import oracle
from oracle import ed
from oracle.dual import DualIsing


@pytest.mark.parametrize("order", [1, 2])
def test_scan_equals_dual_ising_image(order):
    """2+1D: U_p <-> tau^x_p, sigma^x_l <-> tau^z tau^z; the projected Z ground state maps
    onto tau^x = +1 everywhere.  The Ising image is an independent implementation."""
    lat = oracle.Lattice(2, (2, 3))
    n_pts, sub, g_f, t_s = 8, 5, 2.0, 0.4
    loops = [lat.plaq[0], lat.rect_loop(0, 0, 1, 2, 1)]
    got = oracle.adiabatic_scan(lat, oracle.zground_state(lat), g_f, n_pts, sub, t_s, order,
                                loops=loops)
    du = DualIsing(lat.plaq, lat.N)
    phi = np.full(1 << du.n, 1 / np.sqrt(1 << du.n), dtype=np.complex128)
    dt, cx, cz = oracle.schedule_coupling_ramp(t_s * n_pts, n_pts * sub, 0.0, g_f)
    # the 1x2 rectangle encloses plaquettes 0 and the one next to it along x
    encl = [p for p in range(len(lat.plaq))
            if set(int(q) for q in lat.plaq[p]) & set(int(q) for q in loops[1])]
    for k in range(n_pts):
        sl = slice(k * sub, (k + 1) * sub)
        phi = du.evolve(phi, dt, cx[sl], cz[sl], order)
        z = -sum(du.expect_tx(phi, [p]) for p in range(du.n))
        x = -sum(du.expect_bond(phi, l) for l in range(lat.N))
        assert got[k, 0] == pytest.approx(cx[sl][-1], abs=0)
        assert abs(got[k, 2] - z) < 1e-11
        assert abs(got[k, 3] - x) < 1e-11
        assert abs(got[k, 4] - 1.0) < 1e-12
        assert abs(got[k, 5] - du.expect_tx(phi, [0])) < 1e-11
    assert len(encl) >= 2


def test_scan_pure_z_is_stationary():
    """g = 0: the projected Z ground state only picks up a phase, <Z> = -N_p throughout."""
    lat = oracle.Lattice(2, (2, 2))
    psi0 = oracle.zground_state(lat)
    x0 = -sum(oracle.expect_x(psi0, lat.N, [q]) for q in range(lat.N))
    rows = oracle.adiabatic_scan(lat, psi0, 0.0, 6, 4, 0.5, 2)
    assert np.allclose(rows[:, 2], -len(lat.plaq), atol=1e-12)
    assert np.allclose(rows[:, 3], x0, atol=1e-12)
    assert np.allclose(rows[:, 4], 1.0, atol=1e-12)


def _thooft(lat):
    """V_mu: sigma^x over the mu-links that start on the plane x_mu = 0."""
    out = []
    for mu in range(lat.d):
        links = []
        for s in range(lat.n_sites):
            x, t = [], s
            for nu in range(lat.d):
                x.append(t % lat.L[nu])
                t //= lat.L[nu]
            if x[mu] == 0:
                links.append(lat.d * s + (lat.d - 1 - mu))
        out.append(links)
    return out


def test_scan_follows_ground_energy_and_respects_the_bound():
    """A slow ramp on 2x2: <H(g)> = <Z> + g<X> stays above the exact ground energy of its
    sector (variational bound) and close to it (adiabatic theorem, Sec. 2.2)."""
    lat = oracle.Lattice(2, (2, 2))
    n_pts, sub, g_f, t_s = 20, 20, 2.0, 1.0
    rows = oracle.adiabatic_scan(lat, oracle.zground_state(lat), g_f, n_pts, sub, t_s, 2)
    N = lat.N
    P = ed.sector_projector(N, lat.stars, _thooft(lat))
    for g, _, z, x, _n in rows[:, :5]:
        e0 = ed.sector_spectrum(ed.hamiltonian(N, lat.plaq, g, 1.0), P)[0]
        h = z + g * x
        assert h >= e0 - 1e-9
        assert h - e0 < 0.05
