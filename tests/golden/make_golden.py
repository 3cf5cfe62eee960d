"""Write the stored expected values of the full-length workloads, from the oracle only.

Every number written here comes from ``oracle/`` (the plain FP64 CPU reference); this script
imports nothing from the GPU library.  The workloads are the seeded inputs of ``workloads.py``:

* ``config2_full.json``: the 3x3 torus (18 links), 2000 symmetric steps, T = 100, for each of
  the 21 couplings lambda = 0.1 + 0.095 i: energy, every <U_p>, the 2x2 Wilson loop at each of
  the 9 positions, every <G_i>, every <sigma^x_l>, the norm.
* ``config3_full_lam<lambda>.json``: the 2x2x2 torus (24 links), 2000 symmetric steps, T = 100,
  one file per coupling (each takes about half an hour on eight host cores): energy, every
  <U_p>, <sigma^x_l>, <G_i>, the three non-contractible Wilson lines through site 0, the
  Z and X densities of states (Sec. 3.3), the norm.

H(s) = -lambda sum sigma^x - s sum U_p with s = j/n at the right end of step j (Sec. 2.2),
start |+>^N, expectations divided by the norm (Sec. 2.4).

* ``config5_dual.json``: the 4x4 torus (32 links), 1000 symmetric steps, T = 50, lambda in
  {0.5, 1.0, 1.5}: every <U_p> and <sigma^x_l> from the exact Wegner-dual image.

Usage: python tests/golden/make_golden.py config2
       python tests/golden/make_golden.py config5
       python tests/golden/make_golden.py config3 [lambda ...]
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import workloads  # noqa: E402


def _run(lat, w, lam):
    dt, cx, cz = oracle.schedule_plaquette_ramp(w.T, w.n_steps, lam, 1.0)
    psi = oracle.plus_state(lat.N)
    oracle.evolve(psi, lat, dt, cx, cz, w.order)
    return psi, float(cx[-1]), float(cz[-1])


def config2():
    w = workloads.CONFIG2
    lat = oracle.Lattice(w.d, w.L)
    out = {"_about": "3x3 torus, 2000 symmetric Trotter steps, T = 100, start |+>^18, "
                     "H(s) = -lambda sum sigma^x - s sum U_p, s = j/n (Sec. 2.2, eq. (s)); "
                     "written by tests/golden/make_golden.py from the FP64 oracle only",
           "workload": w.name, "results": {}}
    w22 = [lat.rect_loop(lat.site((x, y)), 0, 1, 2, 2) for y in range(3) for x in range(3)]
    for lam in w.lambdas:
        t0 = time.time()
        psi, cxf, czf = _run(lat, w, lam)
        r = oracle.readout(psi, lat, cxf, czf)
        wl = [oracle.expect_z(psi, lat.N, lp) for lp in w22]
        out["results"][repr(lam)] = {
            "lambda": lam, "energy": r["energy"], "norm": r["norm"], "plaq": list(r["plaq"]),
            "sigma_x": list(r["sigma_x"]), "stars": list(r["stars"]),
            "gauss_violation": r["gauss_violation"], "w22": wl,
            "w22_mean": float(np.mean(wl))}
        print(f"config2 lambda={lam:.3f} done in {time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, "config2_full.json"), "w") as fh:
        json.dump(out, fh, indent=1)


def config3(lams):
    w = workloads.CONFIG3
    lat = oracle.Lattice(w.d, w.L)
    lines = [[int(q) for q in lat.line(0, mu)] for mu in range(lat.d)]
    for lam in lams:
        t0 = time.time()
        psi, cxf, czf = _run(lat, w, lam)
        r = oracle.readout(psi, lat, cxf, czf)
        res = {"_about": "2x2x2 torus, 2000 symmetric Trotter steps, T = 100, start |+>^24, "
                         "H(s) = -lambda sum sigma^x - s sum U_p, s = j/n (Sec. 2.2, eq. (s)); "
                         "Z and X densities of states as in Sec. 3.3 (index m: Z = 2m - N_p, "
                         "index k: X = 2k - N_l); written by tests/golden/make_golden.py from "
                         "the FP64 oracle only",
               "workload": w.name, "lambda": lam, "energy": r["energy"], "norm": r["norm"],
               "plaq": list(r["plaq"]), "sigma_x": list(r["sigma_x"]),
               "stars": list(r["stars"]), "gauss_violation": r["gauss_violation"],
               "plaq_mean": float(np.mean(r["plaq"])),
               "wilson_lines": {"links": lines,
                                "values": [oracle.expect_z(psi, lat.N, ln) for ln in lines]},
               "zdos": list(oracle.zdos(psi, lat)), "xdos": list(oracle.xdos(psi, lat.N)),
               "oracle_seconds": time.time() - t0}
        with open(os.path.join(HERE, f"config3_full_lam{lam}.json"), "w") as fh:
            json.dump(res, fh, indent=1)
        print(f"config3 lambda={lam} done in {time.time() - t0:.1f} s", flush=True)


def config5():
    """4x4 torus (32 links), 1000 symmetric steps, T = 50, lambda in {0.5, 1.0, 1.5}: every
    <U_p> and <sigma^x_l> from the exact Wegner-dual image (2^16 amplitudes, oracle/dual.py),
    the full state being too large for the host."""
    from oracle.dual import DualIsing
    w = workloads.CONFIG5
    lat = oracle.Lattice(w.d, w.L)
    D = DualIsing(lat.plaq, lat.N)
    out = {"_about": "4x4 torus, 1000 symmetric Trotter steps, T = 50, start |+>^32, "
                     "H(s) = -lambda sum sigma^x - s sum U_p, s = j/n (Sec. 2.2, eq. (s)); "
                     "<U_p> and <sigma^x_l> of the exact Wegner-dual transverse-field Ising "
                     "image (oracle/dual.py); written by tests/golden/make_golden.py from the "
                     "oracle only", "workload": w.name, "results": {}}
    for lam in w.lambdas:
        t0 = time.time()
        dt, cx, cz = oracle.schedule_plaquette_ramp(w.T, w.n_steps, lam, 1.0)
        phi = D.evolve(D.ghz(), dt, cx, cz, w.order)
        plaq = [D.expect_tx(phi, [p]) for p in range(lat.n_plaq)]
        sx = [D.expect_bond(phi, q) for q in range(lat.N)]
        out["results"][repr(lam)] = {"lambda": lam, "plaq": plaq, "sigma_x": sx,
                                     "energy": float(-cx[-1] * np.sum(sx) - cz[-1] * np.sum(plaq))}
        print(f"config5 lambda={lam} done in {time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, "config5_dual.json"), "w") as fh:
        json.dump(out, fh, indent=1)


if __name__ == "__main__":
    what = sys.argv[1] if len(sys.argv) > 1 else "config2"
    if what == "config2":
        config2()
    elif what == "config5":
        config5()
    elif what == "config3":
        lams = [float(x) for x in sys.argv[2:]] or list(workloads.CONFIG3.lambdas)
        config3(lams)
    else:
        raise SystemExit("usage: make_golden.py config2 | config5 | config3 [lambda ...]")
