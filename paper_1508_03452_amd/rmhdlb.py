"""Thin ctypes binding of the C ABI in include/rmhdlb.h.

Argument marshalling only: every step of the method runs in the HIP library
(librmhdlb.so).  PyTorch provides the device memory (each context's workspace
is a torch tensor of rmhdlb_workspace_bytes) and the stream.  If the library
is missing this module raises; there is no other code path.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librmhdlb.so")

RMHDLB_OK, RMHDLB_EINVAL, RMHDLB_ENOMEM, RMHDLB_EDEVICE, RMHDLB_ERECOVERY, RMHDLB_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
RMHDLB_ESTATE, RMHDLB_ELIMIT = -6, -7
NOALLOC_MAX_SAMPLES = 1 << 20
BC = {"periodic": 0, "open": 1, "driven": 2}
STORAGE = {"f64": 0, "f32": 1, "f16": 2}
OUT_FIELDS = ("n", "p", "eps", "ux", "uy", "uz", "Ex", "Ey", "Ez", "Bx", "By", "Bz", "Jx", "Jy", "Jz", "rho_c")

_dp = ctypes.POINTER(ctypes.c_double)


class rmhdlb_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("bc_lo", ctypes.c_int32 * 3), ("bc_hi", ctypes.c_int32 * 3),
        ("dx", ctypes.c_double), ("c", ctypes.c_double), ("mu0", ctypes.c_double),
        ("tau", ctypes.c_double), ("tau_h", ctypes.c_double), ("alpha", ctypes.c_double),
        ("Gamma", ctypes.c_double), ("sigma", ctypes.c_double), ("nu", ctypes.c_double),
        ("storage", ctypes.c_int32), ("divb_fix", ctypes.c_int32), ("null_band", ctypes.c_int32),
        ("collision", ctypes.c_int32), ("flux", ctypes.c_int32), ("b_prev", ctypes.c_int32),
        ("reserved", ctypes.c_int32 * 2), ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
    ]


class rmhdlb_fields_in(ctypes.Structure):
    _fields_ = [("n", _dp), ("p", _dp), ("u", _dp * 3), ("E", _dp * 3), ("B", _dp * 3), ("rho_c", _dp)]


class rmhdlb_fields_out(ctypes.Structure):
    _fields_ = [("n", _dp), ("p", _dp), ("eps", _dp), ("u", _dp * 3), ("E", _dp * 3), ("B", _dp * 3),
                ("J", _dp * 3), ("rho_c", _dp)]


class rmhdlb_diag(ctypes.Structure):
    _fields_ = [("energy", ctypes.c_double), ("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
                ("em_energy", ctypes.c_double), ("max_divB", ctypes.c_double), ("charge", ctypes.c_double),
                ("mean_iters", ctypes.c_double), ("recon_rate", ctypes.c_double), ("B0", ctypes.c_double),
                ("null_index", ctypes.c_int64), ("newton_hist", ctypes.c_int64 * 16),
                ("n_failed", ctypes.c_int64), ("n_fallback", ctypes.c_int64), ("step", ctypes.c_int64),
                ("guess_steps", ctypes.c_int64)]


GUESS_PARAMS = 1346


class rmhdlb_guess_weights(ctypes.Structure):
    _fields_ = [("w", ctypes.c_float * GUESS_PARAMS), ("mu_x", ctypes.c_float * 6), ("sd_x", ctypes.c_float * 6),
                ("mu_t", ctypes.c_float * 2), ("sd_t", ctypes.c_float * 2)]


class rmhdlb_train_opts(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int32), ("iters", ctypes.c_int32), ("batch", ctypes.c_int32),
                ("stride", ctypes.c_int32), ("lr", ctypes.c_float), ("reserved", ctypes.c_int32 * 3)]


class rmhdlb_face_in(ctypes.Structure):
    _fields_ = [("n", _dp), ("p", _dp), ("u", _dp * 3), ("B", _dp * 3)]


SYMBOLS = ("rmhdlb_create", "rmhdlb_init_fields", "rmhdlb_step", "rmhdlb_moments", "rmhdlb_destroy",
           "rmhdlb_strerror", "rmhdlb_state_len", "rmhdlb_get_state", "rmhdlb_set_state", "rmhdlb_lattice_tables",
           "rmhdlb_set_driven_face", "rmhdlb_train_guess", "rmhdlb_set_guess_weights", "rmhdlb_set_guess",
           "rmhdlb_guess_samples", "rmhdlb_mlp_eval", "rmhdlb_autotune", "rmhdlb_set_tuning", "rmhdlb_set_force",
           "rmhdlb_batch_create", "rmhdlb_batch_instance", "rmhdlb_batch_step", "rmhdlb_batch_autotune",
           "rmhdlb_batch_set_tuning", "rmhdlb_batch_set_persistent", "rmhdlb_batch_destroy", "rmhdlb_workspace_bytes",
           "rmhdlb_guess_samples_noalloc", "rmhdlb_device_copy")

_LIB = None


def load():
    """Load librmhdlb.so (raises if it has not been built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1508_03452_amd/build.py "
                           "(there is no fallback implementation)")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    L.rmhdlb_create.argtypes = [ctypes.POINTER(rmhdlb_params), vp, ctypes.POINTER(vp)]
    L.rmhdlb_workspace_bytes.argtypes = [ctypes.POINTER(rmhdlb_params)]
    L.rmhdlb_workspace_bytes.restype = ctypes.c_size_t
    L.rmhdlb_init_fields.argtypes = [vp, ctypes.POINTER(rmhdlb_fields_in)]
    L.rmhdlb_step.argtypes = [vp, ctypes.c_int64]
    L.rmhdlb_moments.argtypes = [vp, ctypes.POINTER(rmhdlb_fields_out), ctypes.POINTER(rmhdlb_diag)]
    L.rmhdlb_destroy.argtypes = [vp]
    L.rmhdlb_strerror.argtypes = [ctypes.c_int]
    L.rmhdlb_strerror.restype = ctypes.c_char_p
    L.rmhdlb_state_len.argtypes = [vp]
    L.rmhdlb_state_len.restype = ctypes.c_int64
    L.rmhdlb_get_state.argtypes = [vp, _dp]
    L.rmhdlb_set_state.argtypes = [vp, _dp]
    ip = ctypes.POINTER(ctypes.c_int32)
    L.rmhdlb_lattice_tables.argtypes = [ip, _dp, ip, ip, ip]
    L.rmhdlb_set_driven_face.argtypes = [vp, ctypes.POINTER(rmhdlb_face_in)]
    fp = ctypes.POINTER(ctypes.c_float)
    L.rmhdlb_train_guess.argtypes = [vp, ctypes.POINTER(rmhdlb_train_opts), fp, ctypes.POINTER(rmhdlb_guess_weights),
                                     fp]
    L.rmhdlb_set_guess_weights.argtypes = [vp, ctypes.POINTER(rmhdlb_guess_weights)]
    L.rmhdlb_set_guess.argtypes = [vp, ctypes.c_int32]
    L.rmhdlb_guess_samples.argtypes = [vp, ctypes.c_int32, _dp, _dp]
    L.rmhdlb_guess_samples_noalloc.argtypes = [vp, ctypes.c_int32, _dp, _dp]
    L.rmhdlb_mlp_eval.argtypes = [fp, fp, fp, ctypes.c_int32, fp, fp, fp, vp]
    ip32 = ctypes.POINTER(ctypes.c_int32)
    L.rmhdlb_autotune.argtypes = [vp, ip32, ip32, ip32, ip32]
    L.rmhdlb_set_tuning.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.rmhdlb_set_force.argtypes = [vp, ctypes.POINTER(_dp * 3), ctypes.c_double]
    L.rmhdlb_batch_create.argtypes = [ctypes.POINTER(rmhdlb_params), ctypes.c_int32, vp, ctypes.POINTER(vp)]
    L.rmhdlb_batch_instance.argtypes = [vp, ctypes.c_int32]
    L.rmhdlb_batch_instance.restype = vp
    L.rmhdlb_batch_step.argtypes = [vp, ctypes.c_int64]
    L.rmhdlb_batch_autotune.argtypes = [vp, ip32, ip32, ip32]
    L.rmhdlb_batch_set_tuning.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
    L.rmhdlb_batch_set_persistent.argtypes = [vp, ctypes.c_int32]
    L.rmhdlb_batch_destroy.argtypes = [vp]
    L.rmhdlb_device_copy.argtypes = [vp, vp, ctypes.c_size_t, vp]
    _LIB = L
    return L


def strerror(code):
    return load().rmhdlb_strerror(int(code)).decode()


class RmhdlbError(RuntimeError):
    def __init__(self, code, what):
        super().__init__(f"{what}: {strerror(code)} ({code})")
        self.code = code


def _check(code, what, allow=()):
    if code != RMHDLB_OK and code not in allow:
        raise RmhdlbError(code, what)
    return code


def make_params(shape, bc=None, storage="f64", **kw):
    from .workloads import DEFAULT_PARAMS
    d = dict(DEFAULT_PARAMS)
    d.update(kw)
    P = rmhdlb_params()
    P.nx, P.ny, P.nz = (int(v) for v in shape)
    bc = bc or (("periodic", "periodic"),) * 3
    for a in range(3):
        P.bc_lo[a] = BC[bc[a][0]]
        P.bc_hi[a] = BC[bc[a][1]]
    for k in ("dx", "c", "mu0", "tau", "tau_h", "alpha", "Gamma", "sigma", "nu"):
        setattr(P, k, float(d[k]))
    P.storage = STORAGE[storage] if isinstance(storage, str) else int(storage)
    P.divb_fix = int(d.get("divb_fix", 0))
    P.null_band = int(d.get("null_band", 64))
    P.collision = int(d.get("collision", 0))
    P.flux = int(d.get("flux", 0))
    P.b_prev = int(d.get("b_prev", 0))
    return P


def workspace_bytes(P):
    """Device bytes a context with parameters P needs (0 for invalid parameters)."""
    return int(load().rmhdlb_workspace_bytes(ctypes.byref(P)))


def attach_workspace(P, torch):
    """Allocate the context's device memory as a torch tensor and point P at it; returns the tensor (keep it
    alive as long as the context).  None when P is invalid (rmhdlb_create then reports why)."""
    nbytes = workspace_bytes(P)
    if nbytes == 0:
        return None
    ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    P.workspace = ctypes.c_void_p(ws.data_ptr())
    P.workspace_bytes = nbytes
    return ws


def lattice_tables():
    L = load()
    e = np.zeros(57, dtype=np.int32)
    w = np.zeros(19)
    s, eh, bh = (np.zeros(72, dtype=np.int32) for _ in range(3))
    ip = ctypes.POINTER(ctypes.c_int32)
    _check(L.rmhdlb_lattice_tables(e.ctypes.data_as(ip), w.ctypes.data_as(_dp), s.ctypes.data_as(ip),
                                   eh.ctypes.data_as(ip), bh.ctypes.data_as(ip)), "rmhdlb_lattice_tables")
    return dict(e=e.reshape(19, 3), w=w, s=s.reshape(24, 3), ehat=eh.reshape(24, 3), bhat=bh.reshape(24, 3))


def _dptr(t):
    """Device pointer of a contiguous float64 torch tensor."""
    import torch
    assert t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()
    return ctypes.cast(ctypes.c_void_p(t.data_ptr()), _dp)


def _fptr(t):
    """Device pointer of a contiguous float32 torch tensor (None -> NULL)."""
    import torch
    if t is None:
        return ctypes.POINTER(ctypes.c_float)()
    assert t.dtype == torch.float32 and t.is_cuda and t.is_contiguous()
    return ctypes.cast(ctypes.c_void_p(t.data_ptr()), ctypes.POINTER(ctypes.c_float))


def device_copy(dst, src, stream=None):
    """Copy the bytes of a contiguous CUDA tensor src into dst (same size) with the library's copy kernel."""
    import torch
    nbytes = src.numel() * src.element_size()
    assert dst.numel() * dst.element_size() == nbytes and src.is_contiguous() and dst.is_contiguous()
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(load().rmhdlb_device_copy(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), nbytes,
                                     ctypes.c_void_p(st.cuda_stream)), "rmhdlb_device_copy")


def weights_to_dict(W):
    return dict(w=np.array(list(W.w), dtype=np.float32), mu_x=np.array(list(W.mu_x)), sd_x=np.array(list(W.sd_x)),
                mu_t=np.array(list(W.mu_t)), sd_t=np.array(list(W.sd_t)))


def weights_from_dict(d):
    W = rmhdlb_guess_weights()
    W.w[:] = [float(v) for v in np.asarray(d["w"]).reshape(-1)]
    for k in ("mu_x", "sd_x", "mu_t", "sd_t"):
        getattr(W, k)[:] = [float(v) for v in np.asarray(d[k]).reshape(-1)]
    return W


def mlp_eval(w, X, Yt, stream=None):
    """Forward and backward of the network on a batch (device tensors X: n x 6, Yt: n x 2, float32).
    Returns (Y, grad, loss) as tensors."""
    import torch
    n = X.shape[0]
    Y = torch.empty((n, 2), dtype=torch.float32, device="cuda")
    g = torch.empty(GUESS_PARAMS, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    wh = np.ascontiguousarray(np.asarray(w, dtype=np.float32))
    st = stream if stream is not None else torch.cuda.current_stream()
    _check(load().rmhdlb_mlp_eval(wh.ctypes.data_as(ctypes.POINTER(ctypes.c_float)), _fptr(X.contiguous()),
                                  _fptr(Yt.contiguous()), int(n), _fptr(Y), _fptr(g), _fptr(loss),
                                  ctypes.c_void_p(st.cuda_stream)), "rmhdlb_mlp_eval")
    return Y, g, loss


class Solver:
    """One rmhdlb context on the current torch device and stream.  shape = (nx, ny, nz).
    workspace: "torch" (default) allocates the context's device memory as a torch tensor and passes it to
    rmhdlb_create; "library" lets the library allocate it."""

    def __init__(self, shape, bc=None, storage="f64", stream=None, _handle=None, workspace="torch", **params):
        import torch
        self.torch = torch
        self.shape = tuple(int(v) for v in shape)
        nx, ny, nz = self.shape
        self.grid = (nz, ny, nx)
        self.P = make_params(self.shape, bc, storage, **params)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._owned = _handle is None
        self.workspace = None
        if _handle is not None:   # an instance owned by a Batch
            self._h = ctypes.c_void_p(_handle)
            return
        if workspace == "torch":
            self.workspace = attach_workspace(self.P, torch)
        elif workspace != "library":
            raise ValueError(f"workspace must be 'torch' or 'library', not {workspace!r}")
        self._h = ctypes.c_void_p()
        _check(load().rmhdlb_create(ctypes.byref(self.P), ctypes.c_void_p(self.stream.cuda_stream),
                                    ctypes.byref(self._h)), "rmhdlb_create")

    def close(self):
        if getattr(self, "_h", None) and self._h.value and getattr(self, "_owned", True):
            load().rmhdlb_destroy(self._h)
        self._h = ctypes.c_void_p()

    def autotune(self):
        """Time the launch shapes and keep the fastest: (px, zb, zg, yw)."""
        px, zb, zg, yw = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().rmhdlb_autotune(self._h, ctypes.byref(px), ctypes.byref(zb), ctypes.byref(zg),
                                      ctypes.byref(yw)), "rmhdlb_autotune")
        return int(px.value), int(zb.value), int(zg.value), int(yw.value)

    def set_tuning(self, px, zb, zg=1, yw=1):
        _check(load().rmhdlb_set_tuning(self._h, int(px), int(zb), int(zg), int(yw)), "rmhdlb_set_tuning")

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _dev(self, a):
        torch = self.torch
        if isinstance(a, torch.Tensor):
            t = a.to(device="cuda", dtype=torch.float64)
        else:
            t = torch.from_numpy(np.array(np.broadcast_to(np.asarray(a, dtype=np.float64), self.grid)))
            t = t.to("cuda")
        return t.reshape(self.grid).contiguous()

    def init_fields(self, fields):
        """fields: n, p, u (3), E (3), B (3), rho_c (None => Gauss) as numpy arrays or tensors."""
        keep = {k: self._dev(fields[k]) for k in ("n", "p")}
        fin = rmhdlb_fields_in()
        fin.n, fin.p = _dptr(keep["n"]), _dptr(keep["p"])
        for k in ("u", "E", "B"):
            ts = [self._dev(x) for x in fields[k]]
            keep[k] = ts
            setattr(fin, k, (_dp * 3)(*[_dptr(t) for t in ts]))
        if fields.get("rho_c") is not None:
            keep["rho_c"] = self._dev(fields["rho_c"])
            fin.rho_c = _dptr(keep["rho_c"])
        else:
            fin.rho_c = _dp()
        _check(load().rmhdlb_init_fields(self._h, ctypes.byref(fin)), "rmhdlb_init_fields")
        self.stream.synchronize()   # inputs are borrowed only for the call
        return self

    def set_driven_face(self, face):
        """Prescribed fields of the driven low-z face: n, p, u (3), B (3), each (ny, nx)."""
        nx, ny, _ = self.shape
        torch = self.torch

        def dev(a):
            if isinstance(a, torch.Tensor):
                return a.to(device="cuda", dtype=torch.float64).reshape(ny, nx).contiguous()
            return torch.from_numpy(np.array(np.broadcast_to(np.asarray(a, dtype=np.float64), (ny, nx)))).to("cuda")
        keep = [dev(face["n"]), dev(face["p"])]
        u = [dev(x) for x in face["u"]]
        B = [dev(x) for x in face["B"]]
        fin = rmhdlb_face_in()
        fin.n, fin.p = _dptr(keep[0]), _dptr(keep[1])
        fin.u = (_dp * 3)(*[_dptr(t) for t in u])
        fin.B = (_dp * 3)(*[_dptr(t) for t in B])
        _check(load().rmhdlb_set_driven_face(self._h, ctypes.byref(fin)), "rmhdlb_set_driven_face")
        self.stream.synchronize()   # inputs are borrowed only for the call
        return self

    def train_guess(self, init_w, n_samples, iters, batch=512, lr=3e-3, stride=7919):
        """Train the learned recovery guess on cells of the current state; installs it and returns
        (weights dict, losses)."""
        o = rmhdlb_train_opts()
        o.n_samples, o.iters, o.batch, o.stride, o.lr = int(n_samples), int(iters), int(batch), int(stride), float(lr)
        w0 = np.ascontiguousarray(np.asarray(init_w, dtype=np.float32))
        W = rmhdlb_guess_weights()
        losses = np.zeros(max(int(iters), 1), dtype=np.float32)
        fp = ctypes.POINTER(ctypes.c_float)
        _check(load().rmhdlb_train_guess(self._h, ctypes.byref(o), w0.ctypes.data_as(fp), ctypes.byref(W),
                                         losses.ctypes.data_as(fp)), "rmhdlb_train_guess")
        return weights_to_dict(W), losses[:int(iters)]

    def set_force(self, F, gate=0.0):
        """External force density F = (Fx, Fy, Fz) on the grid (numpy or tensors), or None to switch it off;
        it acts while the previous step's largest |beta| is below gate (<= 0: always)."""
        if F is None:
            _check(load().rmhdlb_set_force(self._h, None, 0.0), "rmhdlb_set_force")
            return
        keep = [self._dev(a) for a in F]
        ptrs = (_dp * 3)(*[_dptr(t) for t in keep])
        _check(load().rmhdlb_set_force(self._h, ctypes.byref(ptrs), float(gate)), "rmhdlb_set_force")
        self.stream.synchronize()   # the copies read the temporaries above

    def set_guess_weights(self, d):
        _check(load().rmhdlb_set_guess_weights(self._h, ctypes.byref(weights_from_dict(d))), "rmhdlb_set_guess_weights")

    def set_guess(self, on):
        _check(load().rmhdlb_set_guess(self._h, 1 if on else 0), "rmhdlb_set_guess")

    def guess_samples(self, n_samples, noalloc=False):
        """Features and targets of sampled cells (the learned guess's training data); noalloc uses the
        entry point that allocates no device memory (n_samples <= NOALLOC_MAX_SAMPLES)."""
        torch = self.torch
        F = torch.empty((n_samples, 6), dtype=torch.float64, device="cuda")
        T = torch.empty((n_samples, 2), dtype=torch.float64, device="cuda")
        fn = load().rmhdlb_guess_samples_noalloc if noalloc else load().rmhdlb_guess_samples
        rc = _check(fn(self._h, int(n_samples), _dptr(F), _dptr(T)), fn.__name__, allow=(RMHDLB_ERECOVERY,))
        return F, T, rc

    def step(self, nsteps=1):
        _check(load().rmhdlb_step(self._h, int(nsteps)), "rmhdlb_step")

    def moments(self, fields=OUT_FIELDS, diag=True):
        """Primitive fields as cuda tensors (nz, ny, nx) plus a diagnostics dict."""
        torch = self.torch
        outs = {k: torch.empty(self.grid, dtype=torch.float64, device="cuda") for k in fields}
        fo = rmhdlb_fields_out()
        get = lambda k: _dptr(outs[k]) if k in outs else _dp()
        fo.n, fo.p, fo.eps, fo.rho_c = get("n"), get("p"), get("eps"), get("rho_c")
        for base in ("u", "E", "B", "J"):
            setattr(fo, base, (_dp * 3)(*[get(base + a) for a in "xyz"]))
        d = rmhdlb_diag()
        rc = _check(load().rmhdlb_moments(self._h, ctypes.byref(fo), ctypes.byref(d)), "rmhdlb_moments",
                    allow=(RMHDLB_ERECOVERY,))
        res = dict(outs)
        if diag:
            res["diag"] = dict(energy=d.energy, mass=d.mass, momentum=np.array(list(d.momentum)),
                               em_energy=d.em_energy, max_divB=d.max_divB, charge=d.charge,
                               mean_iters=d.mean_iters, n_failed=int(d.n_failed), step=int(d.step),
                               recon_rate=d.recon_rate, null_index=int(d.null_index), B0=d.B0,
                               n_fallback=int(d.n_fallback), guess_steps=int(d.guess_steps),
                               newton_hist=np.array(list(d.newton_hist), dtype=np.int64))
        res["rc"] = rc
        return res

    def state_len(self):
        return int(load().rmhdlb_state_len(self._h))

    def get_state(self):
        t = self.torch.empty(self.state_len(), dtype=self.torch.float64, device="cuda")
        _check(load().rmhdlb_get_state(self._h, _dptr(t)), "rmhdlb_get_state")
        return t.reshape((-1,) + self.grid)

    def set_state(self, state):
        t = self._dev_flat(state)
        _check(load().rmhdlb_set_state(self._h, _dptr(t)), "rmhdlb_set_state")

    def _dev_flat(self, a):
        torch = self.torch
        if isinstance(a, torch.Tensor):
            return a.to(device="cuda", dtype=torch.float64).reshape(-1).contiguous()
        return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64).reshape(-1)).to("cuda")


class Batch:
    """Independent instances stepped together (one launch per step over all of them, replayed from hipGraphs
    on a non-default stream; or, after set_persistent(), each call's steps in one cooperative launch).
    specs: list of (shape, bc, params dict); each instance's device memory is a torch tensor unless
    workspace="library"."""

    def __init__(self, specs, storage="f32", stream=None, workspace="torch"):
        import torch
        self.torch = torch
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        n = len(specs)
        arr = (rmhdlb_params * n)()
        self.workspaces = []
        for i, (shape, bc, params) in enumerate(specs):
            arr[i] = make_params(shape, bc, storage, **params)
            if workspace == "torch":
                self.workspaces.append(attach_workspace(arr[i], torch))
        self._h = ctypes.c_void_p()
        _check(load().rmhdlb_batch_create(arr, n, ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(self._h)),
               "rmhdlb_batch_create")
        self.instances = [Solver(shape, bc, storage, self.stream, _handle=load().rmhdlb_batch_instance(self._h, i),
                                 **params) for i, (shape, bc, params) in enumerate(specs)]

    def step(self, nsteps=1):
        _check(load().rmhdlb_batch_step(self._h, int(nsteps)), "rmhdlb_batch_step")

    def autotune(self):
        """Time the batch's tile shapes and occupancies and keep the fastest: (px, yw, waves)."""
        px, yw, wv = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(load().rmhdlb_batch_autotune(self._h, ctypes.byref(px), ctypes.byref(yw), ctypes.byref(wv)),
               "rmhdlb_batch_autotune")
        return int(px.value), int(yw.value), int(wv.value)

    def set_tuning(self, px, yw=1, waves=2):
        _check(load().rmhdlb_batch_set_tuning(self._h, int(px), int(yw), int(waves)), "rmhdlb_batch_set_tuning")

    def set_persistent(self, on=True):
        """Step each call in one cooperative launch of the persistent kernel (on) or by graph replays (off)."""
        _check(load().rmhdlb_batch_set_persistent(self._h, 1 if on else 0), "rmhdlb_batch_set_persistent")

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            for s in self.instances:
                s._h = ctypes.c_void_p()
            load().rmhdlb_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
