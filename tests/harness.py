"""Helpers shared by the GPU tests: run the HIP library and the oracle on the same inputs."""
from __future__ import annotations

import contextlib

import numpy as np

import oracle
from paper_1910_08020_amd import lgt

CDT = {lgt.LGT_C64: np.complex64, lgt.LGT_C128: np.complex128}


@contextlib.contextmanager
def gpu_ctx(d, L, dtype=lgt.LGT_C128, state=None):
    ctx = lgt.lgt_create(d, list(L), 1, dtype)
    try:
        if state is not None:
            lgt.lgt_set_state(ctx, np.ascontiguousarray(state, dtype=CDT[dtype]))
        yield ctx
    finally:
        lgt.lgt_destroy(ctx)


def get_state(ctx) -> np.ndarray:
    info = lgt.lgt_info(ctx)
    return lgt.lgt_get_state(ctx, info["state_bytes"], CDT[info["dtype"]]).astype(np.complex128)


def gpu_evolve(d, L, dtype, T, n, h_x, h_p, order, form=lgt.LGT_FORM_FUSED, state=None,
               first=0, count=None, ramp=lgt.LGT_RAMP_PLAQ, g0=0.0, g1=0.0):
    with gpu_ctx(d, L, dtype, state) as ctx:
        s = lgt.make_schedule(T, n, h_x, h_p, ramp=ramp, g0=g0, g1=g1)
        lgt.lgt_evolve(ctx, s, order, form, first, count)
        return get_state(ctx)


def oracle_evolve(lat, T, n, h_x, h_p, order, state=None, first=0, count=None,
                  form="fused"):
    dt, cx, cz = oracle.schedule_plaquette_ramp(T, n, h_x, h_p)
    if count is None:
        count = n - first
    psi = oracle.plus_state(lat.N) if state is None else np.array(state, dtype=np.complex128)
    return oracle.evolve(psi, lat, dt, cx[first:first + count], cz[first:first + count], order,
                         form=form)


def infidelity(a, b) -> float:
    na, nb = np.vdot(a, a).real, np.vdot(b, b).real
    return float(1.0 - abs(np.vdot(a, b)) ** 2 / (na * nb))
