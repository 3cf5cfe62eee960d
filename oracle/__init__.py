"""Plain FP64 CPU oracle for the Trotterized adiabatic Z2 lattice-gauge evolution.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the GPU library (``paper_1910_08020_amd``) and never imports it.

The heavy loops live in ``lgt_oracle.c`` (plain C, FP64); this module wraps
them with ctypes and adds the pieces that follow directly from the paper's
formulas:

* the stepwise schedule of Sec. 2.2 (``g_{k,m} = (k-1) g_s + m delta``: the
  coupling of a substep is taken at its right end), in the paper's form
  ``H = Z + g X`` and in the form ``H(s) = -h_x sum sigma^x - s h_p sum U_p``
  where the plaquette coefficient ramps instead;
* expectation values normalised as <psi|O|psi>/<psi|psi> (Sec. 2.4).

Each function names the passage it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lgt_oracle.c")
_LIB = os.path.join(_HERE, "liblgt_oracle.so")

_c_int_p = ctypes.POINTER(ctypes.c_int)
_c_dbl_p = ctypes.POINTER(ctypes.c_double)
_c_u64_p = ctypes.POINTER(ctypes.c_uint64)


def build(force: bool = True) -> str:
    """Compile the C oracle with gcc (FP64, no fast-math, OpenMP loops)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp",
               "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        L.orc_counts.argtypes = [ctypes.c_int, _c_int_p, _c_int_p, _c_int_p, _c_int_p]
        L.orc_plaquettes.argtypes = [ctypes.c_int, _c_int_p, _c_int_p]
        L.orc_stars.argtypes = [ctypes.c_int, _c_int_p, _c_int_p]
        L.orc_walk_links.argtypes = [ctypes.c_int, _c_int_p, ctypes.c_int, _c_int_p,
                                     ctypes.c_int, _c_int_p]
        L.orc_init_plus.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_init_basis.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64]
        L.orc_rx_link.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.orc_x_layer.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double]
        L.orc_plaq_layer.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_int_p,
                                     ctypes.c_double]
        for name in ("orc_evolve", "orc_evolve_circuit"):
            f = getattr(L, name)
            f.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_int_p,
                          ctypes.c_longlong, _c_dbl_p, _c_dbl_p, ctypes.c_double,
                          ctypes.c_int]
            f.restype = ctypes.c_int
        L.orc_cnot.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_rz.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.orc_rx.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double]
        L.orc_plaq_gadget.argtypes = [ctypes.c_void_p, ctypes.c_int, _c_int_p, ctypes.c_double]
        L.orc_cz.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int]
        L.orc_project_zero.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]
        L.orc_anc_gadget.argtypes = [ctypes.c_void_p, ctypes.c_int, _c_int_p, ctypes.c_int,
                                     ctypes.c_double]
        L.orc_evolve_ancilla.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_int_p,
                                         ctypes.c_longlong, _c_dbl_p, _c_dbl_p, ctypes.c_double,
                                         ctypes.c_int, ctypes.c_int]
        L.orc_evolve_ancilla.restype = ctypes.c_int
        L.orc_prepare_ground_circuit.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                                 _c_int_p]
        L.orc_norm2.argtypes = [ctypes.c_void_p, ctypes.c_int]
        L.orc_norm2.restype = ctypes.c_double
        L.orc_expect_z.argtypes = [ctypes.c_void_p, ctypes.c_int, _c_int_p, ctypes.c_int]
        L.orc_expect_z.restype = ctypes.c_double
        L.orc_expect_x.argtypes = [ctypes.c_void_p, ctypes.c_int, _c_int_p, ctypes.c_int]
        L.orc_expect_x.restype = ctypes.c_double
        L.orc_zdos.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, _c_int_p, _c_dbl_p]
        L.orc_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.orc_uniform.restype = ctypes.c_double
        L.orc_sample.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint64,
                                 ctypes.c_uint64, _c_u64_p]
        L.orc_sample.restype = ctypes.c_int
        L.orc_cdf.argtypes = [ctypes.c_void_p, ctypes.c_int, _c_dbl_p]
        _lib = L
    return _lib


def _ip(a: np.ndarray):
    return a.ctypes.data_as(_c_int_p)


def _dp(a: np.ndarray):
    return a.ctypes.data_as(_c_dbl_p)


def _state_arg(psi: np.ndarray, N: int):
    if psi.dtype != np.complex128 or not psi.flags.c_contiguous or psi.size != (1 << N):
        raise ValueError("state must be a contiguous complex128 array of 2^N amplitudes")
    return psi.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# lattice (Sec. 2.1 and the caption of Fig. 1)
# ---------------------------------------------------------------------------
class Lattice:
    """Periodic d-dimensional lattice, d in {2, 3}; links carry the qubits."""

    def __init__(self, d: int, L):
        L = list(L)
        if len(L) != d:
            raise ValueError("need one extent per dimension")
        self.d = d
        self.L = L
        Lc = np.asarray(L, dtype=np.int32)
        ns, nl, npq = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        if lib().orc_counts(d, _ip(Lc), ctypes.byref(ns), ctypes.byref(nl),
                            ctypes.byref(npq)) != 0:
            raise ValueError("unsupported lattice")
        self.n_sites, self.n_links, self.n_plaq = ns.value, nl.value, npq.value
        self.plaq = np.zeros((self.n_plaq, 4), dtype=np.int32)
        lib().orc_plaquettes(d, _ip(Lc), _ip(self.plaq))
        self.stars = np.zeros((self.n_sites, 2 * d), dtype=np.int32)
        lib().orc_stars(d, _ip(Lc), _ip(self.stars))
        self._Lc = Lc

    @property
    def N(self) -> int:
        return self.n_links

    def walk(self, start_site: int, moves) -> np.ndarray:
        """Links of a closed walk; moves are +-(mu+1) (a Wegner-Wilson contour)."""
        mv = np.asarray(moves, dtype=np.int32)
        out = np.zeros(len(mv), dtype=np.int32)
        k = lib().orc_walk_links(self.d, _ip(self._Lc), start_site, _ip(mv), len(mv), _ip(out))
        if k < 0:
            raise ValueError("bad walk")
        return out[:k].copy()

    def rect_loop(self, start_site: int, mu: int, nu: int, a: int, b: int) -> np.ndarray:
        """Boundary of an a x b rectangle in the (mu, nu) plane, walked counter-clockwise."""
        moves = [mu + 1] * a + [nu + 1] * b + [-(mu + 1)] * a + [-(nu + 1)] * b
        return self.walk(start_site, moves)

    def line(self, start_site: int, mu: int) -> np.ndarray:
        """Non-contractible loop C_mu: L_mu links straight along mu (Sec. 2.1)."""
        return self.walk(start_site, [mu + 1] * self.L[mu])

    def contour(self, k: int) -> np.ndarray:
        """The Wegner-Wilson contours c1, c2, c3 of Sec. 3.1 (perimeters 4 : 6 : 8, areas
        1 : 2 : 3) as closed walks from site 0.  2D: the unit square, the 1 x 2 rectangle
        along x, the L of three squares (one on top of the second).  3D (the contour figure
        is missing; a planar 1 x 2 rectangle would wrap around an extent of 2): the xy
        square, then bent up the xz face along its x edge, then across the xy face one step
        up in z."""
        walks2 = {1: [1, 2, -1, -2], 2: [1, 1, 2, -1, -1, -2], 3: [1, 1, 2, 2, -1, -2, -1, -2]}
        walks3 = {1: [1, 2, -1, -2], 2: [2, 1, -2, 3, -1, -3], 3: [2, 1, -2, 3, 2, -1, -2, -3]}
        return self.walk(0, (walks2 if self.d == 2 else walks3)[k])

    def thooft(self, mu: int) -> list:
        """Links of the 't Hooft operator V_mu (sigma^x string, Sec. 2.1): the mu-links of
        the sites with coordinate x_mu = 0, which pierce one closed dual surface."""
        out = []
        for s in range(self.n_sites):
            x, t = [], s
            for nu in range(self.d):
                x.append(t % self.L[nu])
                t //= self.L[nu]
            if x[mu] == 0:
                out.append(self.d * s + (self.d - 1 - mu))
        return out

    def site(self, x) -> int:
        s, stride = 0, 1
        for mu in range(self.d):
            s += (x[mu] % self.L[mu]) * stride
            stride *= self.L[mu]
        return s


# ---------------------------------------------------------------------------
# schedule (Sec. 2.2)
# ---------------------------------------------------------------------------
def schedule_plaquette_ramp(T: float, n_steps: int, h_x: float, h_p: float,
                            midpoint: bool = False):
    """H_j = -h_x sum sigma^x - s_j h_p sum U_p, s_j = j/n (right end of step j).

    The right-end rule mirrors g_{k,m} = (k-1) g_s + m delta of Sec. 2.2: the
    first substep already uses delta and the last one uses the final value.
    Returns (dt, cx[n], cz[n]).
    """
    j = np.arange(1, n_steps + 1, dtype=np.float64)
    s = (j - 0.5) / n_steps if midpoint else j / n_steps
    dt = T / n_steps
    cx = np.full(n_steps, float(h_x))
    cz = s * float(h_p)
    return dt, cx, cz


def schedule_coupling_ramp(T: float, n_steps: int, g0: float, g1: float,
                           midpoint: bool = False):
    """The paper's form H = Z + g X = -sum U_p - g sum sigma^x, g from g0 to g1.

    Substep j (1-based) uses g_j = g0 + (g1 - g0) j / n, the same right-end
    rule as g_{k,m} = (k-1) g_s + m delta with g_s = (g1-g0) n_sub / n.
    """
    j = np.arange(1, n_steps + 1, dtype=np.float64)
    f = (j - 0.5) / n_steps if midpoint else j / n_steps
    dt = T / n_steps
    cx = g0 + (g1 - g0) * f
    cz = np.ones(n_steps)
    return dt, cx, cz


# ---------------------------------------------------------------------------
# states and evolution
# ---------------------------------------------------------------------------
def plus_state(N: int) -> np.ndarray:
    psi = np.empty(1 << N, dtype=np.complex128)
    lib().orc_init_plus(_state_arg(psi, N), N)
    return psi


def basis_state(N: int, b0: int) -> np.ndarray:
    psi = np.empty(1 << N, dtype=np.complex128)
    lib().orc_init_basis(_state_arg(psi, N), N, b0)
    return psi


def evolve(psi: np.ndarray, lat: Lattice, dt: float, cx, cz, order: int,
           form: str = "fused") -> np.ndarray:
    """In-place Trotterized evolution, eq. (a) (order 1) or eq. (s) (order 2)."""
    N = lat.N
    cx = np.ascontiguousarray(cx, dtype=np.float64)
    cz = np.ascontiguousarray(cz, dtype=np.float64)
    if cx.shape != cz.shape:
        raise ValueError("cx and cz must have one entry per step")
    f = lib().orc_evolve if form == "fused" else lib().orc_evolve_circuit
    rc = f(_state_arg(psi, N), N, lat.n_plaq, _ip(lat.plaq), len(cx), _dp(cx), _dp(cz),
           float(dt), int(order))
    if rc != 0:
        raise ValueError("bad order")
    return psi


def x_layer(psi, N, alpha):
    lib().orc_x_layer(_state_arg(psi, N), N, float(alpha))
    return psi


def plaq_layer(psi, lat: Lattice, theta):
    lib().orc_plaq_layer(_state_arg(psi, lat.N), lat.N, lat.n_plaq, _ip(lat.plaq), float(theta))
    return psi


def cnot(psi, N, c, t):
    lib().orc_cnot(_state_arg(psi, N), N, c, t)
    return psi


def rz(psi, N, q, phi):
    lib().orc_rz(_state_arg(psi, N), N, q, float(phi))
    return psi


def rx(psi, N, q, phi):
    lib().orc_rx(_state_arg(psi, N), N, q, float(phi))
    return psi


def cz_gate(psi, Ntot, a, b):
    lib().orc_cz(_state_arg(psi, Ntot), Ntot, a, b)
    return psi


def project_zero(psi, Ntot, q):
    lib().orc_project_zero(_state_arg(psi, Ntot), Ntot, q)
    return psi


# ---------------------------------------------------------------------------
# one ancilla qubit on bit N of an (N+1)-qubit state (Sec. 2.2 eq. (ara), Sec. 2.3,
# and the controlled evolution of Sec. 2.4)
# ---------------------------------------------------------------------------
def anc_gadget(psi, Ntot, links, a, theta):
    """eq. (ara) for one plaquette: CNOTs from its links onto ancilla a, R_z^a(-2 theta),
    the CNOTs in reverse order."""
    ln = np.ascontiguousarray(links, dtype=np.int32)
    lib().orc_anc_gadget(_state_arg(psi, Ntot), Ntot, _ip(ln), int(a), float(theta))
    return psi


def with_ancilla(psi_lattice: np.ndarray, anc: int = 0) -> np.ndarray:
    """|psi> (x) |anc>_a with the ancilla on the new top bit."""
    out = np.zeros(2 * psi_lattice.size, dtype=np.complex128)
    off = psi_lattice.size if anc else 0
    out[off:off + psi_lattice.size] = psi_lattice
    return out


def evolve_ancilla(psi: np.ndarray, lat: Lattice, dt: float, cx, cz, order: int,
                   controlled: bool = False) -> np.ndarray:
    """In-place evolution of an (N+1)-qubit state in the ancilla circuit form: eq. (ara)
    for each plaquette, R_x on each link, in the orders of eq. (a) / eq. (s).  With
    `controlled`, every R_x sits between two CZ(ancilla, link): the ancilla then sets the
    direction of time for both parts, the U(t) of the phase-estimation passage."""
    N = lat.N
    cx = np.ascontiguousarray(cx, dtype=np.float64)
    cz = np.ascontiguousarray(cz, dtype=np.float64)
    if cx.shape != cz.shape:
        raise ValueError("cx and cz must have one entry per step")
    rc = lib().orc_evolve_ancilla(_state_arg(psi, N + 1), N, lat.n_plaq, _ip(lat.plaq),
                                  len(cx), _dp(cx), _dp(cz), float(dt), int(order),
                                  1 if controlled else 0)
    if rc != 0:
        raise ValueError("bad order")
    return psi


def prepare_ground_circuit(lat: Lattice) -> np.ndarray:
    """Sec. 2.3 with the ancilla: |+>^N |0>_a, then for every plaquette CNOTs onto the
    ancilla, a measurement selecting ancilla |0>, CNOTs back; normalised at the end."""
    N = lat.N
    psi = with_ancilla(plus_state(N), 0)
    lib().orc_prepare_ground_circuit(_state_arg(psi, N + 1), N, lat.n_plaq, _ip(lat.plaq))
    return psi / np.sqrt(norm2(psi, N + 1))


# ---------------------------------------------------------------------------
# observables (Sec. 2.4): normalised expectations, norm reported separately
# ---------------------------------------------------------------------------
def norm2(psi, N) -> float:
    return lib().orc_norm2(_state_arg(psi, N), N)


def raw_z(psi, N, links) -> float:
    ln = np.ascontiguousarray(links, dtype=np.int32)
    return lib().orc_expect_z(_state_arg(psi, N), N, _ip(ln), len(ln))


def raw_x(psi, N, links) -> float:
    ln = np.ascontiguousarray(links, dtype=np.int32)
    return lib().orc_expect_x(_state_arg(psi, N), N, _ip(ln), len(ln))


def expect_z(psi, N, links) -> float:
    """<prod_{l in links} sigma^z_l>: a Wegner-Wilson loop or a plaquette U_p."""
    return raw_z(psi, N, links) / norm2(psi, N)


def expect_x(psi, N, links) -> float:
    """<prod_{l in links} sigma^x_l>: a single link, a Gauss star G_i, a 't Hooft loop."""
    return raw_x(psi, N, links) / norm2(psi, N)


def zdos(psi, lat: Lattice) -> np.ndarray:
    """D(z) of Sec. 3.3, indexed by m = number of odd plaquettes (z = 2m - N_p)."""
    out = np.zeros(lat.n_plaq + 1)
    lib().orc_zdos(_state_arg(psi, lat.N), lat.N, lat.n_plaq, _ip(lat.plaq), _dp(out))
    return out / norm2(psi, lat.N)


def xdos(psi: np.ndarray, N: int) -> np.ndarray:
    """D(x) of Sec. 3.3: weights |<c_x|psi>|^2 of the sigma^x eigenstates |c_x> (link l at
    sigma^x = +1 for c_l = 0, -1 for c_l = 1), binned by k = popcount(c), X = 2k - N.
    <c_x|b> = 2^(-N/2) (-1)^(b.c): a Hadamard on every link, written out per link."""
    phi = np.array(psi, dtype=np.complex128)
    r = 1.0 / np.sqrt(2.0)
    for q in range(N):
        v = phi.reshape(-1, 2, 1 << q)
        a0 = v[:, 0, :].copy()
        a1 = v[:, 1, :].copy()
        v[:, 0, :] = (a0 + a1) * r
        v[:, 1, :] = (a0 - a1) * r
    c = np.arange(1 << N, dtype=np.uint64)
    pop = np.zeros(1 << N, dtype=np.int64)
    for q in range(N):
        pop += ((c >> np.uint64(q)) & np.uint64(1)).astype(np.int64)
    w = np.abs(phi) ** 2
    return np.bincount(pop, weights=w, minlength=N + 1) / w.sum()


def readout(psi: np.ndarray, lat: Lattice, cx_final: float, cz_final: float) -> dict:
    """The full readout: norm, <U_p>, <sigma^z_l>, <sigma^x_l>, <G_i>, energy.

    Energy follows Sec. 2.4: <H> = -cx sum_l <sigma^x_l> - cz sum_p <U_p>.
    """
    N = lat.N
    n2 = norm2(psi, N)
    plaq = np.array([raw_z(psi, N, p) for p in lat.plaq]) / n2
    sz = np.array([raw_z(psi, N, [q]) for q in range(N)]) / n2
    sx = np.array([raw_x(psi, N, [q]) for q in range(N)]) / n2
    stars = np.array([raw_x(psi, N, s) for s in lat.stars]) / n2
    energy = -cx_final * sx.sum() - cz_final * plaq.sum()
    return {"norm": n2, "plaq": plaq, "sigma_z": sz, "sigma_x": sx, "stars": stars,
            "plaq_sum": plaq.sum(), "energy": energy,
            "gauss_violation": float(np.max(np.abs(1.0 - stars)))}


# ---------------------------------------------------------------------------
# sampling
# ---------------------------------------------------------------------------
def uniform(seed: int, i: int) -> float:
    """Draw i of the counter-based SplitMix64 stream (top 53 bits / 2^53)."""
    return lib().orc_uniform(ctypes.c_uint64(seed), ctypes.c_uint64(i))


def sample(psi, N, n_shots: int, seed: int) -> np.ndarray:
    out = np.zeros(n_shots, dtype=np.uint64)
    rc = lib().orc_sample(_state_arg(psi, N), N, n_shots, ctypes.c_uint64(seed),
                          out.ctypes.data_as(_c_u64_p))
    if rc != 0:
        raise MemoryError("oracle sample")
    return out


def cdf(psi, N) -> np.ndarray:
    out = np.zeros(1 << N)
    lib().orc_cdf(_state_arg(psi, N), N, _dp(out))
    return out


def adiabatic_scan(lat: Lattice, psi0: np.ndarray, g_f: float, n_points: int, substeps: int,
                   t_s: float, order: int, loops=()) -> np.ndarray:
    """The stepwise adiabatic evolution of Sec. 2.2 with a pause after every step.

    H_{k,m} = Z + g_{k,m} X with g_{k,m} = (k-1) g_s + m delta, g_s = g_f / N_s and
    delta = g_s / n: step k is n substeps of length t_s / n, each a first-order (eq. (a))
    or symmetric (eq. (s)) Trotter factor.  After every step the evolution pauses and
    <Z> = -sum_p <U_p>, <X> = -sum_l <sigma^x_l>, the norm and the Wegner-Wilson loops
    <prod_{l in loop} sigma^z_l> are computed (Sec. 3).  Rows: (g, 1, <Z>, <X>, norm,
    loops...), expectations divided by the norm.
    """
    N = lat.N
    total = n_points * substeps
    dt, cx, cz = schedule_coupling_ramp(t_s * n_points, total, 0.0, g_f)
    psi = np.array(psi0, dtype=np.complex128)
    rows = []
    for k in range(n_points):
        sl = slice(k * substeps, (k + 1) * substeps)
        psi = evolve(psi, lat, dt, cx[sl], cz[sl], order)
        n2 = norm2(psi, N)
        z = -sum(raw_z(psi, N, p) for p in lat.plaq) / n2
        x = -sum(raw_x(psi, N, [q]) for q in range(N)) / n2
        w = [raw_z(psi, N, list(loop)) / n2 for loop in loops]
        rows.append([cx[sl][-1], cz[sl][-1], z, x, n2] + w)
    return np.array(rows)


def zground_state(lat: Lattice) -> np.ndarray:
    """prod_p P_p |+>^N normalised, P_p = (1 + U_p)/2 projecting on Z_p = -1 (Sec. 2.3)."""
    N = lat.N
    psi = plus_state(N)
    b = np.arange(1 << N, dtype=np.int64)
    for p in lat.plaq:
        par = np.zeros_like(b)
        for q in p:
            par ^= (b >> int(q)) & 1
        psi = 0.5 * (psi + np.where(par == 1, -1.0, 1.0) * psi)
    return psi / np.sqrt(norm2(np.ascontiguousarray(psi), N))
