"""Oracle for the resistive relativistic MHD lattice Boltzmann step.

TEST INFRASTRUCTURE ONLY.  A plain single-threaded FP64 CPU implementation of
the method (Mohseni, Mendoza, Succi, Herrmann, Sec. III), written in C in the
paper's own variables (``rmhdlb_oracle.c``) and wrapped here with ctypes.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  It shares no code with the HIP library and
never imports it.

Arrays are numpy float64 of shape (nz, ny, nx) (x fastest in memory).
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

FIELDS_OUT = ("n", "p", "eps", "ux", "uy", "uz", "Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz", "rho_c")
BC = {"periodic": 0, "open": 1, "driven": 2}


class _Params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc_lo", ctypes.c_int32 * 3), ("bc_hi", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double), ("c", ctypes.c_double), ("mu0", ctypes.c_double),
        ("tau", ctypes.c_double), ("tau_h", ctypes.c_double),
        ("alpha", ctypes.c_double), ("Gamma", ctypes.c_double), ("sigma", ctypes.c_double),
        ("nu", ctypes.c_double),
        ("divb_fix", ctypes.c_int32), ("null_band", ctypes.c_int32), ("collision", ctypes.c_int32),
        ("flux", ctypes.c_int32), ("b_prev", ctypes.c_int32),
    ]


def lib():
    """Load (building if absent) the oracle library.  With RMHDLB_ORACLE_FMA=1 in the environment the
    process loads the build with contracted multiply-adds instead, which only measures rounding
    sensitivity (see build.py)."""
    global _LIB
    if _LIB is None:
        fma = os.environ.get("RMHDLB_ORACLE_FMA") == "1"
        path = _build.LIB_FMA if fma else _build.LIB
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_build.SRC):
            _build.build(fma=fma)
        L = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        L.rmhdlb_oracle_create.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_void_p)]
        L.rmhdlb_oracle_destroy.argtypes = [ctypes.c_void_p]
        L.rmhdlb_oracle_destroy.restype = None
        L.rmhdlb_oracle_init.argtypes = [ctypes.c_void_p, dp, dp, dp * 3, dp * 3, dp * 3, dp]
        L.rmhdlb_oracle_step.argtypes = [ctypes.c_void_p, ctypes.c_long]
        L.rmhdlb_oracle_moments.argtypes = [ctypes.c_void_p, dp * 16, ctypes.POINTER(ctypes.c_long)]
        L.rmhdlb_oracle_diagnostics.argtypes = [ctypes.c_void_p, dp]
        L.rmhdlb_oracle_get_state.argtypes = [ctypes.c_void_p, dp]
        L.rmhdlb_oracle_set_state.argtypes = [ctypes.c_void_p, dp]
        L.rmhdlb_oracle_state_len.argtypes = [ctypes.c_void_p]
        L.rmhdlb_oracle_state_len.restype = ctypes.c_long
        L.rmhdlb_oracle_lattice.argtypes = [ctypes.POINTER(_Params), ctypes.POINTER(ctypes.c_int), dp, dp, dp, dp,
                                            dp, dp, ctypes.POINTER(ctypes.c_int)]
        L.rmhdlb_oracle_equilibria.argtypes = [ctypes.POINTER(_Params), ctypes.c_double, ctypes.c_double,
                                               ctypes.c_double, dp, dp, dp, dp, dp]
        L.rmhdlb_oracle_h_equilibrium.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, ctypes.c_double, dp]
        L.rmhdlb_oracle_recover.argtypes = [ctypes.POINTER(_Params), dp, ctypes.c_double, dp, dp, dp]
        L.rmhdlb_oracle_ohm.argtypes = [ctypes.POINTER(_Params), dp, dp, dp, ctypes.c_double, dp, dp]
        L.rmhdlb_oracle_set_driven.argtypes = [ctypes.c_void_p, dp, dp, dp * 3, dp * 3]
        L.rmhdlb_oracle_set_force.argtypes = [ctypes.c_void_p, ctypes.POINTER(dp * 3), ctypes.c_double]
        L.rmhdlb_oracle_fluid_tensor.argtypes = [ctypes.c_void_p, dp, dp]
        _LIB = L
    return _LIB


def _ptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _vec(x):
    return np.ascontiguousarray(np.asarray(x, dtype=np.float64).reshape(-1))


DEFAULTS = dict(dx=1.0, c=1.0, mu0=1.0, tau=1.0, tau_h=0.5, alpha=0.1, Gamma=4.0 / 3.0, sigma=1.0,
                nu=27.0 ** 0.5, divb_fix=0, null_band=64, collision=0, flux=0, b_prev=0)


def make_params(shape=(1, 1, 1), bc=None, **kw):
    """shape = (nx, ny, nz); bc = ((lo, hi) per axis) with 'periodic'/'open' ('driven' on the low z face)."""
    d = dict(DEFAULTS)
    d.update(kw)
    P = _Params()
    P.nx, P.ny, P.nz = shape
    bc = bc or (("periodic", "periodic"),) * 3
    for a in range(3):
        P.bc_lo[a] = BC[bc[a][0]]
        P.bc_hi[a] = BC[bc[a][1]]
    for k in ("dx", "c", "mu0", "tau", "tau_h", "alpha", "Gamma", "sigma", "nu"):
        setattr(P, k, float(d[k]))
    P.divb_fix = int(d["divb_fix"])
    P.null_band = int(d["null_band"])
    P.collision = int(d["collision"])
    P.flux = int(d["flux"])
    P.b_prev = int(d["b_prev"])
    return P


class Oracle:
    """One oracle simulation.  ``shape`` is (nx, ny, nz)."""

    def __init__(self, shape, bc=None, **params):
        self.shape = tuple(int(s) for s in shape)
        self.P = make_params(self.shape, bc, **params)
        self._h = ctypes.c_void_p()
        rc = lib().rmhdlb_oracle_create(ctypes.byref(self.P), ctypes.byref(self._h))
        if rc != 0:
            raise ValueError(f"oracle create failed ({rc})")
        nx, ny, nz = self.shape
        self.grid = (nz, ny, nx)

    def __del__(self):
        h = getattr(self, "_h", None)
        if h and h.value and _LIB is not None:
            _LIB.rmhdlb_oracle_destroy(h)
            self._h = None

    def _arr(self, a):
        a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), self.grid))
        return a

    def init(self, fields):
        """fields: n, p, u (3-tuple), E, B, rho_c (None => eps0 div E)."""
        keep = []
        n = self._arr(fields["n"])
        p = self._arr(fields["p"])
        keep += [n, p]
        dp = ctypes.POINTER(ctypes.c_double)
        trip = {}
        for k in ("u", "E", "B"):
            arrs = [self._arr(x) for x in fields[k]]
            keep += arrs
            trip[k] = (dp * 3)(*[_ptr(x) for x in arrs])
        rc_arr = fields.get("rho_c")
        rp = None
        if rc_arr is not None:
            rc_arr = self._arr(rc_arr)
            keep.append(rc_arr)
            rp = _ptr(rc_arr)
        rc = lib().rmhdlb_oracle_init(self._h, _ptr(n), _ptr(p), trip["u"], trip["E"], trip["B"], rp)
        if rc != 0:
            raise ValueError(f"oracle init failed ({rc})")

    def step(self, nsteps=1):
        return lib().rmhdlb_oracle_step(self._h, int(nsteps))

    def moments(self):
        outs = {k: np.empty(self.grid) for k in FIELDS_OUT}
        dp = ctypes.POINTER(ctypes.c_double)
        arr = (dp * 16)(*[_ptr(outs[k]) for k in FIELDS_OUT])
        nf = ctypes.c_long()
        lib().rmhdlb_oracle_moments(self._h, arr, ctypes.byref(nf))
        outs["n_failed"] = int(nf.value)
        return outs

    def diagnostics(self):
        d = np.empty(13)
        lib().rmhdlb_oracle_diagnostics(self._h, _ptr(d))
        return dict(energy=d[0], mass=d[1], momentum=d[2:5].copy(), em_energy=d[5], max_divB=d[6], charge=d[7],
                    n_failed=int(d[8]), mean_iters=d[9], recon_rate=d[10], null_index=int(d[11]), B0=d[12])

    def fluid_tensor(self):
        """Per cell (flattened x fastest): E_f (n,), S (n, 3), Pi (n, 3, 3), N0 (n,) of the recovery of
        the current state, and the recovered eps (n,), beta (n, 3)."""
        n = int(np.prod(self.grid))
        out = np.empty((n, 11))
        rec = np.empty((n, 4))
        lib().rmhdlb_oracle_fluid_tensor(self._h, _ptr(out), _ptr(rec))
        Pi = np.empty((n, 3, 3))
        for (a, b), j in (((0, 0), 4), ((1, 1), 5), ((2, 2), 6), ((0, 1), 7), ((0, 2), 8), ((1, 2), 9)):
            Pi[:, a, b] = Pi[:, b, a] = out[:, j]
        return dict(Ef=out[:, 0].copy(), S=out[:, 1:4].copy(), Pi=Pi, N0=out[:, 10].copy(), eps=rec[:, 0].copy(),
                    beta=rec[:, 1:4].copy())

    def set_driven(self, face):
        """Prescribed fields of the driven low-z face: n, p, u (3-tuple), B (3-tuple), each (ny, nx)."""
        nx, ny, _ = self.shape
        keep = []

        def arr(a):
            a = np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), (ny, nx)))
            keep.append(a)
            return _ptr(a)
        dp = ctypes.POINTER(ctypes.c_double)
        u = (dp * 3)(*[arr(x) for x in face["u"]])
        B = (dp * 3)(*[arr(x) for x in face["B"]])
        rc = lib().rmhdlb_oracle_set_driven(self._h, arr(face["n"]), arr(face["p"]), u, B)
        if rc != 0:
            raise ValueError(f"oracle set_driven failed ({rc})")

    def set_force(self, F, gate=0.0):
        """External force density (Reading R26): F = (Fx, Fy, Fz) arrays on the grid, or None to switch it
        off; it acts while the previous step's largest |beta| is below gate (<= 0: always)."""
        if F is None:
            rc = lib().rmhdlb_oracle_set_force(self._h, None, 0.0)
        else:
            arrs = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.float64), self.grid)) for a in F]
            dp = ctypes.POINTER(ctypes.c_double)
            ptrs = (dp * 3)(*[_ptr(a) for a in arrs])
            rc = lib().rmhdlb_oracle_set_force(self._h, ctypes.byref(ptrs), float(gate))
        if rc != 0:
            raise ValueError(f"oracle set_force failed ({rc})")

    def get_state(self):
        n = lib().rmhdlb_oracle_state_len(self._h)
        out = np.empty(n)
        lib().rmhdlb_oracle_get_state(self._h, _ptr(out))
        return out.reshape((-1,) + self.grid)

    def set_state(self, state):
        s = np.ascontiguousarray(state, dtype=np.float64).reshape(-1)
        assert s.size == lib().rmhdlb_oracle_state_len(self._h)
        lib().rmhdlb_oracle_set_state(self._h, _ptr(s))


# ---- single-cell entry points ------------------------------------------------

def lattice(**params):
    P = make_params(**params)
    e = np.zeros(57, dtype=np.int32)
    w, wp, xi = np.zeros(19), np.zeros(19), np.zeros(76)
    v, ee, bb = np.zeros(72), np.zeros(72), np.zeros(72)
    s = np.zeros(72, dtype=np.int32)
    ip = ctypes.POINTER(ctypes.c_int)
    lib().rmhdlb_oracle_lattice(ctypes.byref(P), e.ctypes.data_as(ip), _ptr(w), _ptr(wp), _ptr(xi), _ptr(v),
                                _ptr(ee), _ptr(bb), s.ctypes.data_as(ip))
    return dict(e=e.reshape(19, 3), w=w, wp=wp, xi=xi.reshape(19, 4), v=v.reshape(24, 3), ee=ee.reshape(24, 3),
                bb=bb.reshape(24, 3), s=s.reshape(24, 3))


def equilibria(eps, p, n, beta, E, B, **params):
    """f_eq (paper variables) and g_eq (paper variables) of one state."""
    P = make_params(**params)
    f, g = np.zeros(19), np.zeros(19)
    lib().rmhdlb_oracle_equilibria(ctypes.byref(P), float(eps), float(p), float(n), _ptr(_vec(beta)),
                                   _ptr(_vec(E)), _ptr(_vec(B)), _ptr(f), _ptr(g))
    return f, g


def h_equilibrium(J, E, B, rho_c, **params):
    P = make_params(**params)
    h = np.zeros(25)
    lib().rmhdlb_oracle_h_equilibrium(ctypes.byref(P), _ptr(_vec(J)), _ptr(_vec(E)), _ptr(_vec(B)),
                                      float(rho_c), _ptr(h))
    return h


def recover(T, N0, Eprev, Bprev, **params):
    """Landau-frame recovery from T^{mu nu} (4x4).  Returns dict or raises."""
    P = make_params(**params)
    out = np.zeros(6)
    T16 = _vec(T)
    it = lib().rmhdlb_oracle_recover(ctypes.byref(P), _ptr(T16), float(N0), _ptr(_vec(Eprev)), _ptr(_vec(Bprev)),
                                     _ptr(out))
    if it < 0:
        raise ArithmeticError("recovery failed")
    return dict(eps=out[0], p=out[1], n=out[2], beta=out[3:6].copy(), iters=it)


def ohm(Eprime, B, u, rho_c, **params):
    P = make_params(**params)
    E, J = np.zeros(3), np.zeros(3)
    lib().rmhdlb_oracle_ohm(ctypes.byref(P), _ptr(_vec(Eprime)), _ptr(_vec(B)), _ptr(_vec(u)), float(rho_c),
                            _ptr(E), _ptr(J))
    return E, J
