"""GPU: the stepwise adiabatic scan with per-step measurement (Sec. 2.2, Sec. 3) against the
oracle, and the paper-size scans against what the paper and the mathematics fix."""
import numpy as np
import pytest

import oracle
from paper_1910_08020_amd import lgt
from tests.harness import gpu_ctx

pytestmark = pytest.mark.gpu

C64, C128 = lgt.LGT_C64, lgt.LGT_C128
TROT, SYM = lgt.LGT_ORDER_TROTTER, lgt.LGT_ORDER_SYMMETRIC


def _mask(links):
    return sum(1 << int(q) for q in links)


def _gpu_scan(d, L, dtype, g_f, n_pts, sub, t_s, order, masks=(), first_point=0):
    with gpu_ctx(d, L, dtype) as ctx:
        lgt.lgt_reset(ctx, lgt.LGT_INIT_ZGROUND, 0)
        s = lgt.make_schedule(t_s * n_pts, n_pts * sub, ramp=lgt.LGT_RAMP_COUPLING, g0=0.0, g1=g_f)
        if first_point:   # the same pauses as the full scan, then resume
            lgt.lgt_scan(ctx, s, order, 0, sub, first_point)
        return lgt.lgt_scan(ctx, s, order, first_point * sub, sub, n_pts - first_point,
                            list(masks))


@pytest.mark.parametrize("order", [TROT, SYM], ids=["trotter", "symmetric"])
def test_scan_matches_oracle_3x3(order):
    lat = oracle.Lattice(2, (3, 3))
    n_pts, sub, g_f, t_s = 10, 6, 2.0, 0.3
    loops = [lat.plaq[0], lat.rect_loop(0, 0, 1, 2, 2)]
    got = _gpu_scan(2, (3, 3), C128, g_f, n_pts, sub, t_s, order, [_mask(x) for x in loops])
    want = oracle.adiabatic_scan(lat, oracle.zground_state(lat), g_f, n_pts, sub, t_s, order,
                                 loops=loops)
    assert got.shape == want.shape
    assert np.max(np.abs(got - want)) < 1e-10
    got32 = _gpu_scan(2, (3, 3), C64, g_f, n_pts, sub, t_s, order, [_mask(x) for x in loops])
    assert np.max(np.abs(got32[:, 2:4] - want[:, 2:4])) < 2e-4
    assert np.max(np.abs(got32[:, 4:] - want[:, 4:])) < 2e-5


def test_scan_matches_oracle_2x2x2():
    lat = oracle.Lattice(3, (2, 2, 2))
    n_pts, sub, g_f, t_s = 2, 3, 2.0, 0.3
    got = _gpu_scan(3, (2, 2, 2), C128, g_f, n_pts, sub, t_s, SYM, [_mask(lat.plaq[5])])
    want = oracle.adiabatic_scan(lat, oracle.zground_state(lat), g_f, n_pts, sub, t_s, SYM,
                                 loops=[lat.plaq[5]])
    assert np.max(np.abs(got - want)) < 1e-10


def test_resumed_scan_equals_the_tail_of_a_full_scan():
    """Pausing is exact: a scan resumed at a step boundary repeats the later rows bit for bit."""
    full = _gpu_scan(2, (3, 3), C64, 2.0, 8, 5, 0.3, SYM)
    tail = _gpu_scan(2, (3, 3), C64, 2.0, 8, 5, 0.3, SYM, first_point=3)
    assert np.array_equal(full[3:], tail)


def test_scan_validation():
    with gpu_ctx(2, (2, 2), C64) as ctx:
        s = lgt.make_schedule(1.0, 10, ramp=lgt.LGT_RAMP_COUPLING, g0=0.0, g1=1.0)
        for args in [(0, 0, 5), (0, 2, 0), (0, 4, 3), (8, 2, 2)]:
            with pytest.raises(lgt.LgtError) as ex:
                lgt.lgt_scan(ctx, s, SYM, *args)
            assert ex.value.status == lgt.LGT_E_INVALID
        with pytest.raises(lgt.LgtError):
            lgt.lgt_scan(ctx, s, SYM, 0, 2, 5, [1 << 9])


def _paper_scan(d, L, order, n, t_s, N_s=2000, g_f=2.0):
    """Sec. 2.6 parameters: g from 0 to 2 in N_s = 2000 steps of g_s = 0.001, each step n
    substeps of t_s / n, from the projected Z ground state, complex64."""
    with gpu_ctx(d, L, C64) as ctx:
        lgt.lgt_reset(ctx, lgt.LGT_INIT_ZGROUND, 0)
        s = lgt.make_schedule(t_s * N_s, n * N_s, ramp=lgt.LGT_RAMP_COUPLING, g0=0.0, g1=g_f)
        return lgt.lgt_scan(ctx, s, order, 0, n, N_s)


def test_paper_scan_3x3_first_order():
    """3x3, first order, n = 500, t_s = 0.02 (Sec. 2.6): the energy stays within the
    adiabatic error of the exact ground energy of the sector (dual Ising, exact
    diagonalisation), never below it, and d2<H>/dg2 bottoms out near the printed
    g_c = 0.380 (Sec. 3.2)."""
    from oracle.dual import DualIsing
    rows = _paper_scan(2, (3, 3), TROT, 500, 0.02)
    g, z, x = rows[:, 0], rows[:, 2], rows[:, 3]
    assert abs(z[0] + 9) < 1e-4
    lat = oracle.Lattice(2, (3, 3))
    du = DualIsing(lat.plaq, lat.N)
    w, V = np.linalg.eigh(du.even_projector())
    B = V[:, w > 0.5]
    for k in range(0, 2000, 50):
        e0 = np.linalg.eigvalsh(B.conj().T @ du.hamiltonian(g[k], 1.0) @ B)[0]
        dev = z[k] + g[k] * x[k] - e0
        assert -1e-3 < dev < 0.05, (g[k], dev)
    gc, _ = lgt.lgt_critical_point(g, z + g * x, stride=10)
    assert 0.36 < gc < 0.41


def test_paper_scan_2x2x2_symmetric():
    """2x2x2, symmetric, n = 200, t_s = 0.1 (Sec. 2.6): <Z> and <X> cross at the self-dual
    point g = 1, <Z>(g) = <X>(1/g) (eq. (dual)), and d2<H>/dg2 bottoms out near the
    printed g_c = 0.986 (Sec. 3.2)."""
    rows = _paper_scan(3, (2, 2, 2), SYM, 200, 0.1)
    g, z, x = rows[:, 0], rows[:, 2], rows[:, 3]
    assert abs(z[0] + 24) < 1e-4
    assert np.max(np.abs(rows[:, 4] - 1)) < 5e-3
    assert 0.99 < lgt.lgt_crossing(g, z, x) < 1.01
    gc, _ = lgt.lgt_critical_point(g, z + g * x, stride=10)
    assert 0.96 < gc < 1.01
    for gq in (0.5, 0.6, 0.7, 0.8, 0.9):
        i, j = int(round(gq * 1000)) - 1, int(round(1000 / gq)) - 1
        assert abs(z[i] - x[j]) < 0.02, gq


@pytest.mark.parametrize("d,L", [(2, (3, 3)), (2, (4, 4)), (3, (2, 2, 2))], ids=["3x3", "4x4", "2x2x2"])
def test_contour_masks_match_oracle(d, L):
    """The Wegner-Wilson contours c1, c2, c3 of Sec. 3.1 (perimeters 4, 6, 8)."""
    lat = oracle.Lattice(d, L)
    with gpu_ctx(d, L, C64) as ctx:
        for k in (1, 2, 3):
            assert lgt.lgt_contour_mask(ctx, k) == _mask(lat.contour(k))
        with pytest.raises(lgt.LgtError) as ex:
            lgt.lgt_contour_mask(ctx, 4)
        assert ex.value.status == lgt.LGT_E_INVALID
    with gpu_ctx(2, (2, 2), C64) as ctx:       # a 1 x 2 block wraps around an extent of 2
        with pytest.raises(lgt.LgtError) as ex:
            lgt.lgt_contour_mask(ctx, 2)
        assert ex.value.status == lgt.LGT_E_UNSUPPORTED


@pytest.mark.parametrize("d,L,n_pts,sub", [(2, (3, 3), 8, 5), (3, (2, 2, 2), 2, 2)],
                         ids=["3x3", "2x2x2"])
def test_contour_scan_matches_oracle(d, L, n_pts, sub):
    lat = oracle.Lattice(d, L)
    loops = [lat.contour(k) for k in (1, 2, 3)]
    got = _gpu_scan(d, L, C128, 2.0, n_pts, sub, 0.3, SYM, [_mask(x) for x in loops])
    want = oracle.adiabatic_scan(lat, oracle.zground_state(lat), 2.0, n_pts, sub, 0.3, SYM,
                                 loops=loops)
    assert np.max(np.abs(got - want)) < 1e-10


def test_wilson_loop_laws_3x3():
    """Sec. 3.1: on the adiabatic state, log<W_c2>/log<W_c1> and log<W_c3>/log<W_c1> start at
    the perimeter ratios 1.5 and 2 (the second-order perturbative result for small g) and
    move towards the area ratios 2 and 3 deep in the confined phase (exact ground state of
    the dual Ising model at g = 2: 1.93 and 2.84).  The paper's 3x3 first-order schedule,
    n = 500, t_s = 0.02, complex64."""
    lat = oracle.Lattice(2, (3, 3))
    with gpu_ctx(2, (3, 3), C64) as ctx:
        masks = [lgt.lgt_contour_mask(ctx, k) for k in (1, 2, 3)]
        lgt.lgt_reset(ctx, lgt.LGT_INIT_ZGROUND, 0)
        s = lgt.make_schedule(0.02 * 2000, 500 * 2000, ramp=lgt.LGT_RAMP_COUPLING, g0=0.0, g1=2.0)
        rows = lgt.lgt_scan(ctx, s, TROT, 0, 500, 2000, masks)
    g, w = rows[:, 0], rows[:, 5:8]
    r2, r3 = np.log(w[:, 1]) / np.log(w[:, 0]), np.log(w[:, 2]) / np.log(w[:, 0])
    small = (g > 0.049) & (g < 0.101)
    assert np.all(np.abs(r2[small] - 1.5) < 0.05) and np.all(np.abs(r3[small] - 2.0) < 0.08)
    assert r2[-1] > 1.8 and r3[-1] > 2.6
    assert lat.n_plaq == 9
