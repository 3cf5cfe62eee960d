"""Pins for the oracle's evolution, readout and sampling.

Every check here compares the oracle against something other than itself:
dense matrix exponentials built from Kronecker products, closed forms,
conservation laws, the Wegner duality to the transverse-field Ising model,
the paper's printed schedule sums and a published RNG stream.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import Lattice, ed
from oracle.dual import DualIsing

L22 = Lattice(2, (2, 2))
L33 = Lattice(2, (3, 3))


def _rand_state(N, seed):
    g = np.random.default_rng(seed)
    v = g.standard_normal(1 << N) + 1j * g.standard_normal(1 << N)
    return v / np.linalg.norm(v)


# --------------------------------------------------------------------------
# single layers and single steps against dense matrix exponentials
# --------------------------------------------------------------------------
def test_x_layer_is_expm():
    N = L22.N
    psi = _rand_state(N, 1)
    a = 0.37
    want = sla.expm(1j * a * ed.h_links(N)) @ psi
    got = oracle.x_layer(psi.copy(), N, a)
    assert np.max(np.abs(got - want)) < 1e-13


def test_plaq_layer_is_expm():
    N = L22.N
    psi = _rand_state(N, 2)
    t = -0.81
    want = sla.expm(1j * t * ed.h_plaq(N, L22.plaq)) @ psi
    got = oracle.plaq_layer(psi.copy(), L22, t)
    assert np.max(np.abs(got - want)) < 1e-13


@pytest.mark.parametrize("order", [1, 2])
def test_one_step_is_product_of_expm(order):
    """eq. (a) and eq. (s): order of the factors and signs of the exponents."""
    N = L22.N
    psi = _rand_state(N, 3)
    dt, cx, cz = 0.13, 0.9, 1.7
    want = ed.trotter_step_matrix(N, L22.plaq, dt, cx, cz, order) @ psi
    got = oracle.evolve(psi.copy(), L22, dt, [cx], [cz], order)
    assert np.max(np.abs(got - want)) < 1e-13


@pytest.mark.parametrize("order", [1, 2])
def test_circuit_form_equals_fused_form(order):
    """eq. (ara): the CNOT ladder + R_z gadget reproduces exp(-i t Z_p) exactly."""
    for lat in (L22, L33):
        N = lat.N
        psi = _rand_state(N, 4)
        dt, cx, cz = oracle.schedule_plaquette_ramp(1.0, 6, 0.8, 1.1)
        a = oracle.evolve(psi.copy(), lat, dt, cx, cz, order, form="fused")
        b = oracle.evolve(psi.copy(), lat, dt, cx, cz, order, form="circuit")
        assert np.max(np.abs(a - b)) < 1e-13


def test_gate_definitions():
    """R_z(phi) = exp(-i sigma^z phi/2), R_x(phi) = exp(-i sigma^x phi/2), CNOT (Sec. 2.2)."""
    N = 3
    psi = _rand_state(N, 5)
    phi = 0.6
    assert np.allclose(oracle.rz(psi.copy(), N, 1, phi),
                       ed.op_on(N, 1, sla.expm(-0.5j * phi * ed.SZ)) @ psi, atol=1e-14)
    assert np.allclose(oracle.rx(psi.copy(), N, 2, phi),
                       ed.op_on(N, 2, sla.expm(-0.5j * phi * ed.SX)) @ psi, atol=1e-14)
    C = np.zeros((8, 8))
    for b in range(8):
        c = b ^ (4 if b & 1 else 0)     # control qubit 0, target qubit 2
        C[c, b] = 1
    assert np.allclose(oracle.cnot(psi.copy(), N, 0, 2), C @ psi, atol=1e-15)


# --------------------------------------------------------------------------
# Trotter error scaling against the piecewise-exact stepwise evolution
# --------------------------------------------------------------------------
def _trotter_errors(order, ns):
    N = L22.N
    errs = []
    for n in ns:
        dt, cx, cz = oracle.schedule_plaquette_ramp(5.0, n, 1.0, 1.0)
        psi0 = oracle.plus_state(N)
        exact = ed.exact_stepwise(psi0, N, L22.plaq, dt, cx, cz)
        got = oracle.evolve(psi0.copy(), L22, dt, cx, cz, order)
        errs.append(np.linalg.norm(got - exact))
    return np.array(errs)


def test_first_order_error_halves():
    """eq. (asymtotal): total error ~ t_s^2/n per unit time, i.e. linear in dt."""
    e = _trotter_errors(1, [50, 100, 200, 400])
    r = e[:-1] / e[1:]
    assert np.all((r > 1.85) & (r < 2.15)), r


def test_symmetric_error_quarters():
    """eq. (total): total error ~ t_s^3/n^2 per unit time, i.e. quadratic in dt."""
    e = _trotter_errors(2, [50, 100, 200, 400])
    r = e[:-1] / e[1:]
    assert np.all((r > 3.7) & (r < 4.3)), r


def test_single_step_error_bounds():
    """eq. (error1)/(symmerror): one-step errors scale as tau^2 and tau^3.

    The rigorous first-order bound (tau^2/2)||[Hz, Hx]|| <= 4 g N_p tau^2 holds.
    """
    N = L22.N
    g = 0.7
    Hx = -g * ed.h_links(N)
    Hz = -ed.h_plaq(N, L22.plaq)
    e1, e2 = [], []
    taus = [0.04, 0.02, 0.01]
    for tau in taus:
        U = sla.expm(-1j * tau * (Hx + Hz))
        A = ed.trotter_step_matrix(N, L22.plaq, tau, g, 1.0, 1)
        S = ed.trotter_step_matrix(N, L22.plaq, tau, g, 1.0, 2)
        e1.append(np.linalg.norm(U - A, 2))
        e2.append(np.linalg.norm(U - S, 2))
        assert e1[-1] <= 4 * g * L22.n_plaq * tau ** 2
    assert 3.6 < e1[0] / e1[1] < 4.4 and 3.6 < e1[1] / e1[2] < 4.4
    assert 7.2 < e2[0] / e2[1] < 8.8 and 7.2 < e2[1] / e2[2] < 8.8
    # the ED matrices and the oracle agree on every column
    psi = _rand_state(N, 6)
    got = oracle.evolve(psi.copy(), L22, taus[0], [g], [1.0], 1)
    A = ed.trotter_step_matrix(N, L22.plaq, taus[0], g, 1.0, 1)
    assert np.max(np.abs(got - A @ psi)) < 1e-13


# --------------------------------------------------------------------------
# closed forms
# --------------------------------------------------------------------------
@pytest.mark.parametrize("order", [1, 2])
def test_no_plaquette_term_precession(order):
    """h_p = 0 from |0...0>: every link precesses, <sigma^z_l>(t) = cos(2 h_x t)."""
    N = L22.N
    h_x, T, n = 0.9, 3.0, 40
    dt, cx, cz = oracle.schedule_plaquette_ramp(T, n, h_x, 0.0)
    psi = oracle.basis_state(N, 0)
    oracle.evolve(psi, L22, dt, cx, cz, order)
    for q in range(N):
        assert abs(oracle.expect_z(psi, N, [q]) - np.cos(2 * h_x * T)) < 1e-13


@pytest.mark.parametrize("order", [1, 2])
def test_no_link_term_pure_phase(order):
    """h_x = 0: the evolution is diagonal, psi_b(T) = psi_b(0) exp(i h_p sum_j dt s_j u(b)).

    With s_j = j/n, sum_j dt s_j = dt (n+1)/2; u(b) = sum_p u_p(b) from the ED matrix.
    """
    N = L22.N
    h_p, T, n = 1.3, 2.0, 25
    dt, cx, cz = oracle.schedule_plaquette_ramp(T, n, 0.0, h_p)
    psi0 = _rand_state(N, 7)
    got = oracle.evolve(psi0.copy(), L22, dt, cx, cz, order)
    u = np.real(np.diag(ed.h_plaq(N, L22.plaq)))
    want = psi0 * np.exp(1j * h_p * dt * (n + 1) / 2 * u)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("order", [1, 2])
def test_midpoint_rule_pure_phase(order):
    """The midpoint option s_j = (j - 1/2)/n with h_x = 0: sum_j dt s_j = dt n / 2 = T / 2
    exactly, so psi_b(T) = psi_b(0) exp(i h_p (T/2) u(b)).  The right-end rule of Sec. 2.2
    gives dt (n+1)/2 instead, so a schedule on the wrong rule fails by h_p dt / 2."""
    N = L22.N
    h_p, T, n = 1.3, 2.0, 25
    dt, cx, cz = oracle.schedule_plaquette_ramp(T, n, 0.0, h_p, midpoint=True)
    psi0 = _rand_state(N, 8)
    got = oracle.evolve(psi0.copy(), L22, dt, cx, cz, order)
    u = np.real(np.diag(ed.h_plaq(N, L22.plaq)))
    want = psi0 * np.exp(1j * h_p * T / 2 * u)
    assert np.max(np.abs(got - want)) < 1e-12
    # the coupling ramp on the midpoint rule: sum_j g_j = n (g0 + g1) / 2, so with only the
    # link term (cz dropped by a zero plaquette weight) |0...0> precesses by the mean coupling
    dt, cx, cz = oracle.schedule_coupling_ramp(T, n, 0.4, 1.6, midpoint=True)
    psi = oracle.evolve(oracle.basis_state(N, 0), L22, dt, cx, 0.0 * cz, order)
    for q in range(N):
        assert abs(oracle.expect_z(psi, N, [q]) - np.cos(2 * 1.0 * T)) < 1e-12


def _h_apply(psi, N, plaq, cx, cz):
    """H psi for H = -cx sum_l sigma^x_l - cz sum_p U_p, each Pauli factor applied by
    reshaping the amplitude array around its qubit axis (bit q of the index is qubit q)."""
    out = np.zeros_like(psi)
    for q in range(N):
        v = psi.reshape(1 << (N - 1 - q), 2, 1 << q)
        out -= cx * v[:, ::-1, :].reshape(-1)
    for p in plaq:
        w = psi.copy()
        for q in p:
            v = w.reshape(1 << (N - 1 - int(q)), 2, 1 << int(q))
            v[:, 1, :] *= -1
        out -= cz * w
    return out


@pytest.mark.parametrize("d,L", [(2, (2, 2)), (2, (2, 3))], ids=["2x2", "2x3"])
def test_readout_energy_matches_exact_expectation(d, L):
    """readout(): energy = <psi|H|psi>/<psi|psi> for random (unnormalised) states, with H
    built from Pauli factors (a dense Kronecker matrix on 2x2), and every reported
    observable against its operator: <U_p>, <sigma^x_l>, <sigma^z_l>, <G_i>, the norm."""
    lat = Lattice(d, L)
    N = lat.N
    for seed, (cx, cz) in ((11, (0.7, 1.3)), (12, (-1.9, 0.4)), (13, (2.5, -0.8))):
        psi = 1.7 * _rand_state(N, seed)
        r = oracle.readout(psi, lat, cx, cz)
        n2 = np.vdot(psi, psi).real
        if N <= 8:
            H = ed.hamiltonian(N, lat.plaq, cx, cz)
            want = np.vdot(psi, H @ psi).real / n2
        else:
            want = np.vdot(psi, _h_apply(psi, N, lat.plaq, cx, cz)).real / n2
        assert abs(r["energy"] - want) < 1e-12 * max(1.0, abs(want))
        assert abs(r["norm"] - n2) < 1e-12 * n2
        if N <= 8:
            for p, v in zip(lat.plaq, r["plaq"]):
                assert abs(v - np.vdot(psi, ed.pauli_product(N, p, ed.SZ) @ psi).real / n2) < 1e-13
            for q in range(N):
                assert abs(r["sigma_x"][q] - np.vdot(psi, ed.op_on(N, q, ed.SX) @ psi).real / n2) < 1e-13
                assert abs(r["sigma_z"][q] - np.vdot(psi, ed.op_on(N, q, ed.SZ) @ psi).real / n2) < 1e-13
            for s, v in zip(lat.stars, r["stars"]):
                assert abs(v - np.vdot(psi, ed.pauli_product(N, s, ed.SX) @ psi).real / n2) < 1e-13
    # an eigenstate: the energy of |+>^N under the link term alone is -cx N
    r = oracle.readout(oracle.plus_state(N), lat, 0.9, 0.0)
    assert abs(r["energy"] + 0.9 * N) < 1e-12


def test_plus_state_stationary_without_plaquettes():
    """|+>^N is an eigenstate of sum sigma^x: only a global phase e^{i N h_x T}."""
    N = L33.N
    dt, cx, cz = oracle.schedule_plaquette_ramp(1.0, 10, 0.7, 0.0)
    psi = oracle.evolve(oracle.plus_state(N), L33, dt, cx, cz, 1)
    want = np.exp(1j * N * 0.7 * 1.0) / np.sqrt(1 << N)
    assert np.max(np.abs(psi - want)) < 1e-12


def test_schedule_sums_match_paper():
    """Sec. 2.2: sum g_{k,m} = (N_s^2 n + N_s) g_s / 2, and the printed sum of g^2."""
    for Ns, n, gs in ((20, 5, 0.1), (2000, 200, 0.001), (7, 13, 0.3)):
        dt, cx, cz = oracle.schedule_coupling_ramp(Ns * 1.0, Ns * n, 0.0, Ns * gs)
        assert abs(cx[0] - gs / n) < 1e-15 and abs(cx[-1] - Ns * gs) < 1e-12
        s1 = 0.5 * (Ns * Ns * n + Ns) * gs
        s2 = ((Ns - 1) * Ns * (2 * Ns - 1) * n * gs ** 2 / 6
              + Ns * n * (n + 1) * (2 * n + 1) * gs ** 2 / (6 * n * n)
              + Ns * (Ns - 1) * (n + 1) * gs ** 2 / 2)
        assert abs(cx.sum() - s1) < 1e-9 * s1
        assert abs((cx ** 2).sum() - s2) < 1e-9 * s2
        assert np.all(cz == 1.0)


# --------------------------------------------------------------------------
# exact invariants (Sec. 2.1, 2.3, 3.5)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("order", [1, 2])
def test_invariants_3x3(order):
    lat = L33
    N = lat.N
    dt, cx, cz = oracle.schedule_plaquette_ramp(3.0, 60, 0.6, 1.0)
    psi = oracle.evolve(oracle.plus_state(N), lat, dt, cx, cz, order)
    r = oracle.readout(psi, lat, cx[-1], cz[-1])
    assert abs(r["norm"] - 1) < 1e-11
    assert r["gauss_violation"] < 1e-12                      # G_i = 1
    assert np.max(np.abs(r["sigma_z"])) < 1e-12               # no magnetisation (Sec. 3.5)
    for mu in range(2):                                       # <W_mu> = 0 on non-contractible loops
        assert abs(oracle.expect_z(psi, N, lat.line(0, mu))) < 1e-12
    # Gauss law also holds for the individual star operator on a random site
    assert abs(oracle.expect_x(psi, N, lat.stars[4]) - 1) < 1e-12


def test_invariants_3d():
    lat = Lattice(3, (2, 2, 2))
    N = lat.N
    dt, cx, cz = oracle.schedule_plaquette_ramp(0.2, 2, 1.0, 1.0)
    psi = oracle.evolve(oracle.plus_state(N), lat, dt, cx, cz, 2)
    assert abs(oracle.norm2(psi, N) - 1) < 1e-12
    for s in range(lat.n_sites):
        assert abs(oracle.expect_x(psi, N, lat.stars[s]) - 1) < 1e-12
    for q in (0, 5, 23):
        assert abs(oracle.expect_z(psi, N, [q])) < 1e-12


# --------------------------------------------------------------------------
# 2+1D Wegner duality (Sec. 3.2): exact image on the dual Ising model
# --------------------------------------------------------------------------
@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("lat", [L22, L33], ids=["2x2", "3x3"])
def test_evolution_equals_dual_ising(order, lat):
    N = lat.N
    dt, cx, cz = oracle.schedule_plaquette_ramp(4.0, 80, 0.8, 1.0)
    psi = oracle.evolve(oracle.plus_state(N), lat, dt, cx, cz, order)
    D = DualIsing(lat.plaq, N)
    phi = D.evolve(D.ghz(), dt, cx, cz, order)
    for p in range(lat.n_plaq):
        assert abs(oracle.expect_z(psi, N, lat.plaq[p]) - D.expect_tx(phi, [p])) < 1e-11
    for l in range(N):
        assert abs(oracle.expect_x(psi, N, [l]) - D.expect_bond(phi, l)) < 1e-11
    if lat is L33:
        # a 2x2 Wilson loop is the product of the tau^x of its four plaquettes
        w = lat.rect_loop(0, 0, 1, 2, 2)
        inside = [lat.site([x, y]) for x in range(2) for y in range(2)]   # plaquette index = site
        assert abs(oracle.expect_z(psi, N, w) - D.expect_tx(phi, inside)) < 1e-11


@pytest.mark.parametrize("g", [0.3, 1.0, 2.5])
def test_duality_spectrum(g):
    """H(g) = g H~(1/g): the gauge theory in the G=1, V=(+,+) sector has the spectrum
    of g times the even-sector transverse-field Ising model at coupling 1/g."""
    lat = L22
    N = lat.N
    H = ed.hamiltonian(N, lat.plaq, g, 1.0)           # Z + g X
    lines = []
    for mu in range(2):      # 't Hooft loops: mu-links starting on x_mu = 0
        links = [2 * s + (1 - mu) for s in range(lat.n_sites)
                 if ([s % 2, s // 2][mu]) == 0]
        lines.append(links)
    P = ed.sector_projector(N, lat.stars, lines)
    e_gauge = ed.sector_spectrum(H, P)
    D = DualIsing(lat.plaq, N)
    e_ising = g * ed.sector_spectrum(D.hamiltonian(1.0, 1.0 / g), D.even_projector())
    assert len(e_gauge) == len(e_ising) == 1 << (lat.n_plaq - 1)
    assert np.max(np.abs(np.sort(e_gauge) - np.sort(e_ising))) < 1e-10


# --------------------------------------------------------------------------
# density of states, sampling
# --------------------------------------------------------------------------
def test_zdos_plus_state_counts():
    """For |+>^N, D(m) = #(basis states with m odd plaquettes) / 2^N (counted from ED)."""
    lat = L33
    N = lat.N
    dos = oracle.zdos(oracle.plus_state(N), lat)
    # eigenvalues of sum U_p on basis states via explicit parity bits
    b = np.arange(1 << N)
    m = np.zeros(1 << N, dtype=np.int64)
    for p in lat.plaq:
        par = np.zeros_like(b)
        for q in p:
            par ^= (b >> int(q)) & 1
        m += par
    want = np.bincount(m, minlength=lat.n_plaq + 1) / (1 << N)
    assert np.max(np.abs(dos - want)) < 1e-14
    assert abs(dos.sum() - 1) < 1e-14


def test_splitmix_stream(golden):
    want = [int(h, 16) for h in golden["splitmix64_seed0"]["outputs_hex"]]
    for i, w in enumerate(want):
        assert oracle.uniform(0, i) == (w >> 11) / 2.0 ** 53


def test_sample_is_inverse_cdf():
    N = 10
    psi = _rand_state(N, 8)
    shots = oracle.sample(psi, N, 4000, 1234)
    p = np.abs(psi) ** 2
    c = np.cumsum(p)
    for i in range(0, 4000, 97):
        u = oracle.uniform(1234, i) * c[-1]
        b = int(shots[i])
        assert c[b] > u and (b == 0 or c[b - 1] <= u)
    # chi^2-style check against the probabilities on coarse bins
    hist = np.bincount(shots.astype(np.int64) >> 6, minlength=16) / 4000
    want = p.reshape(16, 64).sum(axis=1)
    assert np.max(np.abs(hist - want)) < 0.03
