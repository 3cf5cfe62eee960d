"""Ancilla circuits on the GPU (eq. (ara), the controlled evolution of Sec. 2.4 and the
projection circuit of Sec. 2.3) against the oracle, closed forms and the fused path."""
import contextlib

import numpy as np
import pytest

import oracle
from paper_1910_08020_amd import lgt
from tests.harness import CDT, get_state, gpu_evolve

pytestmark = pytest.mark.gpu

C64, C128 = lgt.LGT_C64, lgt.LGT_C128
TROT, SYM = lgt.LGT_ORDER_TROTTER, lgt.LGT_ORDER_SYMMETRIC
ANC, CTL = lgt.LGT_FORM_ANCILLA, lgt.LGT_FORM_CONTROLLED


@contextlib.contextmanager
def anc_ctx(d, L, dtype=C128):
    ctx = lgt.lgt_create_ancilla(d, list(L), 1, dtype)
    try:
        yield ctx
    finally:
        lgt.lgt_destroy(ctx)


def _rand_state(n, seed):
    g = np.random.default_rng(seed)
    v = g.standard_normal(1 << n) + 1j * g.standard_normal(1 << n)
    return v / np.linalg.norm(v)


def test_ancilla_context_layout_and_reset():
    lat = oracle.Lattice(2, (2, 2))
    with anc_ctx(2, (2, 2)) as ctx:
        info = lgt.lgt_info(ctx)
        assert info["n_links"] == lat.N and info["n_qubits"] == lat.N + 1
        assert info["state_bytes"] == 16 << (lat.N + 1)
        want = oracle.with_ancilla(oracle.plus_state(lat.N), 0)
        assert np.max(np.abs(get_state(ctx) - want)) < 1e-15
        lgt.lgt_reset(ctx, lgt.LGT_INIT_BASIS, (1 << lat.N) | 5)
        psi = get_state(ctx)
        assert psi[(1 << lat.N) | 5] == 1 and np.count_nonzero(psi) == 1


@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_gates_match_oracle(dtype):
    """Every gate kind on link qubits and on the ancilla, against the oracle's gates and
    the closed forms of H and X."""
    N = oracle.Lattice(2, (2, 2)).N
    n = N + 1
    psi = _rand_state(n, 3)
    tol = 2e-6 if dtype == C64 else 1e-13
    r2 = 1 / np.sqrt(2)
    b = np.arange(1 << n)
    cases = [(lgt.LGT_GATE_RX, 2, -1, 0.7), (lgt.LGT_GATE_RX, N, -1, -1.1),
             (lgt.LGT_GATE_RZ, 5, -1, 0.3), (lgt.LGT_GATE_RZ, N, -1, 2.2),
             (lgt.LGT_GATE_CNOT, 1, N, 0), (lgt.LGT_GATE_CNOT, N, 6, 0),
             (lgt.LGT_GATE_CZ, N, 3, 0), (lgt.LGT_GATE_CZ, 0, 7, 0),
             (lgt.LGT_GATE_H, N, -1, 0), (lgt.LGT_GATE_H, 4, -1, 0),
             (lgt.LGT_GATE_X, N, -1, 0), (lgt.LGT_GATE_X, 2, -1, 0)]
    with anc_ctx(2, (2, 2), dtype) as ctx:
        for gate, q0, q1, ang in cases:
            lgt.lgt_set_state(ctx, np.ascontiguousarray(psi, dtype=CDT[dtype]))
            lgt.lgt_apply_gate(ctx, gate, q0, q1, ang)
            got = get_state(ctx)
            want = psi.copy()
            if gate == lgt.LGT_GATE_RX:
                oracle.rx(want, n, q0, ang)
            elif gate == lgt.LGT_GATE_RZ:
                oracle.rz(want, n, q0, ang)
            elif gate == lgt.LGT_GATE_CNOT:
                oracle.cnot(want, n, q0, q1)
            elif gate == lgt.LGT_GATE_CZ:
                oracle.cz_gate(want, n, q0, q1)
            elif gate == lgt.LGT_GATE_H:
                lo, hi = psi[(b >> q0) & 1 == 0], psi[(b >> q0) & 1 == 1]
                want[(b >> q0) & 1 == 0] = r2 * (lo + hi)
                want[(b >> q0) & 1 == 1] = r2 * (lo - hi)
            else:
                want = psi[b ^ (1 << q0)]
            assert np.max(np.abs(got - want)) < tol, (gate, q0, q1)


def test_gate_validation():
    with anc_ctx(2, (2, 2)) as ctx:
        n = lgt.lgt_info(ctx)["n_qubits"]
        for args in [(lgt.LGT_GATE_RX, n, -1, 0.1), (lgt.LGT_GATE_CNOT, 1, 1, 0.0),
                     (lgt.LGT_GATE_CZ, 0, n, 0.0), (lgt.LGT_GATE_H, -1, -1, 0.0), (17, 0, 1, 0.0)]:
            with pytest.raises(lgt.LgtError) as e:
                lgt.lgt_apply_gate(ctx, *args)
            assert e.value.status == lgt.LGT_E_INVALID


@pytest.mark.parametrize("order", [TROT, SYM], ids=["trotter", "symmetric"])
@pytest.mark.parametrize("d,L,dtype", [(2, (2, 2), C128), (2, (3, 3), C128), (2, (3, 3), C64)],
                         ids=["2x2-c128", "3x3-c128", "3x3-c64"])
@pytest.mark.parametrize("form,anc", [(ANC, 0), (ANC, 1), (CTL, 0), (CTL, 1), (CTL, 2)],
                         ids=["anc0", "anc1", "ctl0", "ctl1", "ctl+"])
def test_ancilla_forms_match_oracle(d, L, dtype, order, form, anc):
    """The 19-qubit (3x3 + ancilla) and 9-qubit circuits of the paper's ancilla form, with
    the ancilla in |0>, |1> or (controlled only) |+>, against the gate-by-gate oracle."""
    lat = oracle.Lattice(d, L)
    N, n, T = lat.N, 6, 0.3
    dt, cx, cz = oracle.schedule_coupling_ramp(T, n, 0.0, 1.5)
    psi0 = oracle.with_ancilla(oracle.plus_state(N), 0)
    with anc_ctx(d, L, dtype) as ctx:
        if anc == 1:
            lgt.lgt_apply_gate(ctx, lgt.LGT_GATE_X, N)
        elif anc == 2:
            lgt.lgt_apply_gate(ctx, lgt.LGT_GATE_H, N)
        start = get_state(ctx)
        lgt.lgt_evolve(ctx, lgt.make_schedule(T, n, ramp=lgt.LGT_RAMP_COUPLING, g0=0.0, g1=1.5),
                       order, form)
        got = get_state(ctx)
    if anc == 1:
        psi0 = psi0[np.arange(1 << (N + 1)) ^ (1 << N)]
    elif anc == 2:
        psi0 = np.concatenate([psi0[: 1 << N], psi0[: 1 << N]]) / np.sqrt(2)
    assert np.max(np.abs(start - psi0)) < 1e-7
    want = oracle.evolve_ancilla(psi0.copy(), lat, dt, cx, cz, order, controlled=form == CTL)
    rel = 1e-5 if dtype == C64 else 1e-12
    assert np.max(np.abs(got - want)) < rel * np.max(np.abs(want))


@pytest.mark.parametrize("d,L,dtype", [(2, (3, 3), C128), (3, (2, 2, 2), C64)],
                         ids=["3x3-19q", "2x2x2-25q"])
def test_controlled_phase_on_z_ground_state(d, L, dtype):
    """Phase estimation's controlled evolution at g = 0 from (|0> + |1>)/sqrt 2 times the
    Z ground state: <sigma^x_a> = cos(2 E t) with E = -N_p (closed form)."""
    lat = oracle.Lattice(d, L)
    N, n, T = lat.N, 6, 0.18
    with anc_ctx(d, L, dtype) as ctx:
        lgt.lgt_reset(ctx, lgt.LGT_INIT_ZGROUND)
        lgt.lgt_apply_gate(ctx, lgt.LGT_GATE_H, N)
        s = lgt.make_schedule(T, n, cx=np.zeros(n), cz=np.ones(n), ramp=lgt.LGT_RAMP_EXPLICIT)
        lgt.lgt_evolve(ctx, s, SYM, CTL)
        sx = lgt.lgt_measure(ctx, lgt.LGT_OBS_X, masks=[1 << N])[0]
        plaq = lgt.lgt_measure(ctx, lgt.LGT_OBS_PLAQ)[: lat.n_plaq]
    E = -lat.n_plaq
    tol = 2e-5 if dtype == C64 else 1e-11
    assert abs(sx - np.cos(2 * E * T)) < tol
    assert np.max(np.abs(plaq - 1)) < tol


@pytest.mark.parametrize("d,L,dtype", [(2, (3, 3), C128), (3, (2, 2, 2), C64)],
                         ids=["3x3-19q", "2x2x2-25q"])
def test_projection_circuit_equals_z_ground_state(d, L, dtype):
    lat = oracle.Lattice(d, L)
    N = lat.N
    with anc_ctx(d, L, dtype) as ctx:
        lgt.lgt_reset(ctx, lgt.LGT_INIT_ZGROUND_CIRCUIT)
        got = get_state(ctx)
        lgt.lgt_reset(ctx, lgt.LGT_INIT_ZGROUND)
        direct = get_state(ctx)
    tol = 1e-6 if dtype == C64 else 1e-13
    assert np.max(np.abs(got - direct)) < tol
    assert np.max(np.abs(got[1 << N:])) == 0.0
    if N <= 18:
        assert np.max(np.abs(got - oracle.prepare_ground_circuit(lat))) < tol


def test_ancilla_form_25_qubits_equals_fused_path():
    """2x2x2 + ancilla (25 qubits), two symmetric steps: the lattice half equals the fused
    path's state (itself checked against the oracle) and the ancilla half stays empty."""
    n, T = 2, 0.1
    s = lgt.make_schedule(T, n, ramp=lgt.LGT_RAMP_COUPLING, g0=0.0, g1=1.0)
    with anc_ctx(3, (2, 2, 2), C64) as ctx:
        lgt.lgt_evolve(ctx, s, SYM, ANC)
        got = get_state(ctx)
        e = lgt.lgt_measure(ctx, lgt.LGT_OBS_ENERGY, cx=1.0, cz=1.0)[0]
    fused = gpu_evolve(3, (2, 2, 2), C64, T, n, 0.0, 0.0, SYM, ramp=lgt.LGT_RAMP_COUPLING,
                       g0=0.0, g1=1.0)
    N = 24
    assert np.max(np.abs(got[1 << N:])) == 0.0
    assert np.max(np.abs(got[: 1 << N] - fused)) < 1e-5 * np.max(np.abs(fused))
    with contextlib.ExitStack() as st:
        c = lgt.lgt_create(3, [2, 2, 2], 1, C64)
        st.callback(lgt.lgt_destroy, c)
        lgt.lgt_set_state(c, np.ascontiguousarray(fused, dtype=np.complex64))
        e_fused = lgt.lgt_measure(c, lgt.LGT_OBS_ENERGY, cx=1.0, cz=1.0)[0]
    assert abs(e - e_fused) < 1e-5


def test_forms_and_contexts_must_match():
    s = lgt.make_schedule(0.1, 2)
    with anc_ctx(2, (2, 2)) as ctx:
        for form in (lgt.LGT_FORM_FUSED, lgt.LGT_FORM_CIRCUIT):
            with pytest.raises(lgt.LgtError) as e:
                lgt.lgt_evolve(ctx, s, SYM, form)
            assert e.value.status == lgt.LGT_E_UNSUPPORTED
        with pytest.raises(lgt.LgtError) as e:
            lgt.lgt_measure(ctx, lgt.LGT_OBS_XDOS)
        assert e.value.status == lgt.LGT_E_UNSUPPORTED
        with pytest.raises(lgt.LgtError) as e:
            lgt.lgt_tune(ctx, 2)
        assert e.value.status == lgt.LGT_E_UNSUPPORTED
        with pytest.raises(lgt.LgtError) as e:
            lgt.lgt_batch_evolve([ctx], [s], [SYM], 0, 2)
        assert e.value.status == lgt.LGT_E_UNSUPPORTED
    plain = lgt.lgt_create(2, [2, 2], 1, C128)
    try:
        for form in (ANC, CTL):
            with pytest.raises(lgt.LgtError) as e:
                lgt.lgt_evolve(plain, s, SYM, form)
            assert e.value.status == lgt.LGT_E_UNSUPPORTED
        with pytest.raises(lgt.LgtError) as e:
            lgt.lgt_reset(plain, lgt.LGT_INIT_ZGROUND_CIRCUIT)
        assert e.value.status == lgt.LGT_E_UNSUPPORTED
    finally:
        lgt.lgt_destroy(plain)
