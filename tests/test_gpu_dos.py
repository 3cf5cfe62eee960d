"""GPU: densities of states (Sec. 3.3) against the oracle, and the self-duality of the
3+1D theory, D_Z(z, g) = D_X(x = z, 1/g), on the paper-size adiabatic evolution."""
import numpy as np
import pytest

import oracle
import workloads
from paper_1910_08020_amd import lgt
from tests.harness import gpu_ctx

pytestmark = pytest.mark.gpu

C64, C128 = lgt.LGT_C64, lgt.LGT_C128


def _evolved(lat, n=6, lam=0.9):
    dt, cx, cz = oracle.schedule_plaquette_ramp(0.05 * n, n, lam, 1.0)
    return oracle.evolve(oracle.zground_state(lat), lat, dt, cx, cz, 2)


@pytest.mark.parametrize("dtype", [C64, C128], ids=["c64", "c128"])
def test_xdos_and_zdos_match_oracle_3x3(dtype):
    lat = oracle.Lattice(2, (3, 3))
    psi = _evolved(lat)
    tol = 1e-10 if dtype == C128 else 2e-6
    with gpu_ctx(2, (3, 3), dtype, psi) as ctx:
        before = lgt.lgt_get_state(ctx, lgt.lgt_info(ctx)["state_bytes"],
                                   np.complex128 if dtype == C128 else np.complex64)
        xd = lgt.lgt_measure(ctx, lgt.LGT_OBS_XDOS)[: lat.N + 1]
        zd = lgt.lgt_measure(ctx, lgt.LGT_OBS_ZDOS)[: lat.n_plaq + 1]
        after = lgt.lgt_get_state(ctx, lgt.lgt_info(ctx)["state_bytes"], before.dtype)
    assert np.array_equal(before, after)   # measured on a copy
    assert np.max(np.abs(xd - oracle.xdos(psi, lat.N))) < tol
    assert np.max(np.abs(zd - oracle.zdos(psi, lat))) < tol


def test_xdos_matches_oracle_2x2x2_random_state():
    lat = oracle.Lattice(3, (2, 2, 2))
    psi = workloads.random_state(lat.N, stream=17)
    with gpu_ctx(3, (2, 2, 2), C128, psi) as ctx:
        xd = lgt.lgt_measure(ctx, lgt.LGT_OBS_XDOS)[: lat.N + 1]
    assert np.max(np.abs(xd - oracle.xdos(psi, lat.N))) < 1e-10


def test_self_duality_of_the_densities_2x2x2():
    """Sec. 3.3: D_Z(z, g) = D_X(x = z, 1/g) in d = 3, on the adiabatic states of the paper's
    scan (g_s = 0.001, n = 200, t_s = 0.1), at g = 0.8 and 1/g = 1.25; the two densities
    vanish at +-20."""
    n, t_s, g_s = 200, 0.1, 0.001
    k1, k2 = 800, 1250
    with gpu_ctx(3, (2, 2, 2), C64) as ctx:
        lgt.lgt_reset(ctx, lgt.LGT_INIT_ZGROUND, 0)
        s = lgt.make_schedule(t_s * 2000, n * 2000, ramp=lgt.LGT_RAMP_COUPLING, g0=0.0,
                              g1=2000 * g_s)
        lgt.lgt_scan(ctx, s, lgt.LGT_ORDER_SYMMETRIC, 0, n, k1)
        dz = lgt.lgt_measure(ctx, lgt.LGT_OBS_ZDOS)[:25]
        lgt.lgt_scan(ctx, s, lgt.LGT_ORDER_SYMMETRIC, k1 * n, n, k2 - k1)
        dx = lgt.lgt_measure(ctx, lgt.LGT_OBS_XDOS)[:25]
    # both indexed by the eigenvalue 2m - 24
    assert np.max(np.abs(dz - dx)) < 0.02, (dz, dx)
    for arr in (dz, dx):
        assert arr[2] < 1e-6 and arr[22] < 1e-6   # +-20 are forbidden
