"""Pins of the oracle's densities of states (Sec. 3.3)."""
import numpy as np

import oracle
import workloads


def _evolved(lat, n=6, lam=0.9):
    dt, cx, cz = oracle.schedule_plaquette_ramp(0.05 * n, n, lam, 1.0)
    return oracle.evolve(oracle.zground_state(lat), lat, dt, cx, cz, 2)


def test_xdos_mean_is_the_flip_expectation():
    """sum_k (2k - N) D_X(k) = <X> = -sum_l <sigma^x_l>, the latter from pair sums."""
    lat = oracle.Lattice(2, (2, 3))
    psi = workloads.random_state(lat.N, stream=5)
    d = oracle.xdos(psi, lat.N)
    x = -sum(oracle.expect_x(psi, lat.N, [q]) for q in range(lat.N))
    assert abs(np.dot(2 * np.arange(lat.N + 1) - lat.N, d) - x) < 1e-12
    assert abs(d.sum() - 1) < 1e-12


def test_xdos_of_basis_eigenstates():
    """|+>^N sits entirely at X = -N; a basis state spreads binomially."""
    N = 6
    d = oracle.xdos(oracle.plus_state(N), N)
    assert abs(d[0] - 1) < 1e-14 and np.all(np.abs(d[1:]) < 1e-14)
    d = oracle.xdos(oracle.basis_state(N, 0), N)
    binom = np.array([1, 6, 15, 20, 15, 6, 1]) / 64
    assert np.allclose(d, binom, atol=1e-14)


def test_dos_supports_of_gauge_invariant_states(golden):
    """Gauge invariance: sigma^x flips come in closed loops (perimeter 4, 6, ...), so on 3x3
    D_X vanishes off the printed support and at +-14; on 2x2x2 both DOS vanish at +-20."""
    lat = oracle.Lattice(2, (3, 3))
    psi = _evolved(lat)
    d = oracle.xdos(psi, lat.N)
    allowed = set(golden["x_spectrum"]["3x3_superset"])
    for k, w in enumerate(d):
        if 2 * k - lat.N not in allowed:
            assert w < 1e-20, (2 * k - lat.N, w)
    assert d.sum() > 1 - 1e-12
    z = oracle.zdos(psi, lat)
    zs = set(golden["z_spectrum"]["3x3"])
    for m, w in enumerate(z):
        if 2 * m - lat.n_plaq not in zs:
            assert w < 1e-20
