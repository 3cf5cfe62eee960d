"""Pins for the oracle's ancilla circuits: the plaquette gadget of eq. (ara), the
controlled direction of time of the phase-estimation passage (Sec. 2.4) and the
projection circuit of Sec. 2.3.

Each check compares the gate-by-gate oracle with an independent construction: dense
Kronecker-product operators and matrix exponentials, closed forms on eigenstates, and
brute-force counting of the configurations the projections keep.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from oracle import Lattice, ed

L22 = Lattice(2, (2, 2))
L23 = Lattice(2, (2, 3))


def _rand_state(N, seed):
    g = np.random.default_rng(seed)
    v = g.standard_normal(1 << N) + 1j * g.standard_normal(1 << N)
    return v / np.linalg.norm(v)


def _powers(M, n):
    out = np.eye(M.shape[0], dtype=np.complex128)
    for _ in range(n):
        out = M @ out
    return out


@pytest.mark.parametrize("p", [0, 2, 3])
def test_gadget_is_exp_of_plaquette_times_ancilla_z(p):
    """A^-1 R_z^a(-2 theta) A = exp(i theta U_p sigma^z_a): exp(-i theta Z_p) with the
    ancilla in |0>, its inverse with the ancilla in |1> (eq. (ara) and the remark after
    it on the reversed evolution)."""
    N, a, theta = L22.N, L22.N, 0.41
    links = [int(x) for x in L22.plaq[p]]
    psi = _rand_state(N + 1, 10 + p)
    want = sla.expm(1j * theta * ed.pauli_product(N + 1, links + [a], ed.SZ)) @ psi
    got = oracle.anc_gadget(psi.copy(), N + 1, links, a, theta)
    assert np.max(np.abs(got - want)) < 1e-13


def test_gadget_leaves_the_ancilla_where_it_was():
    N, a = L22.N, L22.N
    for anc in (0, 1):
        psi = oracle.with_ancilla(_rand_state(N, 20 + anc), anc)
        for p in L22.plaq:
            oracle.anc_gadget(psi, N + 1, [int(x) for x in p], a, 0.3)
        other = psi[: 1 << N] if anc else psi[1 << N:]
        assert np.max(np.abs(other)) == 0.0


@pytest.mark.parametrize("order", [1, 2])
@pytest.mark.parametrize("lat", [L22, L23], ids=["2x2", "2x3"])
def test_ancilla_zero_is_the_forward_evolution(lat, order):
    """With the ancilla in |0> the ancilla form is the ancilla-free evolution (x) |0>."""
    N, n = lat.N, 7
    dt, cx, cz = oracle.schedule_coupling_ramp(0.35, n, 0.0, 1.3)
    psi = _rand_state(N, 30 + order)
    want = oracle.with_ancilla(oracle.evolve(psi.copy(), lat, dt, cx, cz, order), 0)
    got = oracle.evolve_ancilla(oracle.with_ancilla(psi, 0), lat, dt, cx, cz, order)
    assert np.max(np.abs(got - want)) < 1e-12


@pytest.mark.parametrize("order", [1, 2])
def test_controlled_evolution_is_block_diagonal_in_time_direction(order):
    """U = |0><0| (x) S(dt)^n + |1><1| (x) S(-dt)^n with S the Trotter step of dense
    matrix exponentials (phase-estimation passage, Sec. 2.4)."""
    lat, n, dt, g = L22, 5, 0.09, 0.8
    N = lat.N
    psi = _rand_state(N + 1, 40 + order)
    fwd = _powers(ed.trotter_step_matrix(N, lat.plaq, dt, g, 1.0, order), n)
    bwd = _powers(ed.trotter_step_matrix(N, lat.plaq, -dt, g, 1.0, order), n)
    want = np.concatenate([fwd @ psi[: 1 << N], bwd @ psi[1 << N:]])
    got = oracle.evolve_ancilla(psi.copy(), lat, dt, np.full(n, g), np.ones(n), order,
                                controlled=True)
    assert np.max(np.abs(got - want)) < 1e-12


def test_uncontrolled_ancilla_one_reverses_only_the_plaquette_part():
    """Without the CZ pairs only eq. (ara) follows the ancilla: |1> gives the step with
    cz -> -cz and cx unchanged."""
    lat, n, dt, g = L22, 4, 0.1, 0.7
    N = lat.N
    psi = _rand_state(N, 50)
    M = _powers(ed.trotter_step_matrix(N, lat.plaq, dt, g, -1.0, 2), n)
    got = oracle.evolve_ancilla(oracle.with_ancilla(psi, 1), lat, dt, np.full(n, g),
                                np.ones(n), 2)
    assert np.max(np.abs(got[1 << N:] - M @ psi)) < 1e-12
    assert np.max(np.abs(got[: 1 << N])) == 0.0


@pytest.mark.parametrize("lat", [L22, L23], ids=["2x2", "2x3"])
def test_phase_estimation_phase_on_the_z_ground_state(lat):
    """At g = 0 the Z ground state is an eigenstate with E = -N_p (every U_p = +1).  From
    (|0> + |1>)/sqrt 2 the controlled evolution leaves e^{-iEt}|0> + e^{iEt}|1>, so twice
    the overlap of the two ancilla branches is e^{2iEt}."""
    N, n, dt = lat.N, 6, 0.07
    u = oracle.zground_state(lat)
    psi = np.concatenate([u, u]) / np.sqrt(2)
    oracle.evolve_ancilla(psi, lat, dt, np.zeros(n), np.ones(n), 2, controlled=True)
    E, t = -lat.n_plaq, n * dt
    ov = 2 * np.vdot(psi[: 1 << N], psi[1 << N:])
    assert abs(ov - np.exp(2j * E * t)) < 1e-12


def _gf2_rank(rows):
    rows = [int(r) for r in rows]
    rank = 0
    for bit in range(64):
        piv = next((i for i in range(rank, len(rows)) if (rows[i] >> bit) & 1), None)
        if piv is None:
            continue
        rows[rank], rows[piv] = rows[piv], rows[rank]
        for i in range(len(rows)):
            if i != rank and (rows[i] >> bit) & 1:
                rows[i] ^= rows[rank]
        rank += 1
    return rank


@pytest.mark.parametrize("lat", [L22, L23, Lattice(2, (3, 3))], ids=["2x2", "2x3", "3x3"])
def test_projection_circuit_keeps_the_flat_configurations(lat):
    """Sec. 2.3 with the ancilla: the kept configurations are exactly those with every
    U_p = +1, all with the same amplitude, 2^(N - rank) of them (rank of the plaquette
    parity checks over GF(2)); the ancilla ends in |0>."""
    N = lat.N
    psi = oracle.prepare_ground_circuit(lat)
    assert np.max(np.abs(psi[1 << N:])) == 0.0
    body = psi[: 1 << N]
    masks = [sum(1 << int(q) for q in p) for p in lat.plaq]
    keep = np.ones(1 << N, dtype=bool)
    b = np.arange(1 << N, dtype=np.int64)
    for m in masks:
        par = np.zeros_like(b)
        x = b & m
        while np.any(x):
            par ^= x & 1
            x >>= 1
        keep &= par == 0
    nz = np.abs(body) > 1e-12
    assert np.array_equal(nz, keep)
    assert nz.sum() == 2 ** (N - _gf2_rank(masks))
    assert np.allclose(np.abs(body[nz]), 1 / np.sqrt(nz.sum()), atol=1e-14)
    assert np.max(np.abs(body - oracle.zground_state(lat))) < 1e-13
