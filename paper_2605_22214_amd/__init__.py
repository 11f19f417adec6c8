"""Python binding of libnflbm (the HIP library of the N-component free-energy
lattice Boltzmann update, arXiv 2605.22214) for MI355X / gfx950.

Argument marshalling only: every step of the update runs in the library's HIP
kernels.  The library must have been built (``python -m
paper_2605_22214_amd.build``); importing works without it, but any call that
needs it raises ``RuntimeError`` -- there is no fallback implementation.
"""
import ctypes
import os
import re

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
_ROOT = os.path.dirname(_PKG)
# NFLBM_LIBRARY selects another build of the library (e.g. a development
# build restricted to one component count); by default the in-tree one.
LIB_PATH = os.environ.get("NFLBM_LIBRARY") or os.path.join(_PKG, "libnflbm.so")
HEADER = os.path.join(_ROOT, "include", "nflbm.h")
MAX_COMP = 8

D2Q9, D3Q19 = 0, 1
FP64, FP32, FP16S = 0, 1, 2
FLAG_POTENTIAL_FORCE = 1
FLAG_ALLOW_UNSTABLE = 2
FLAG_G_POPULATIONS = 4
FLAG_NO_HYDRO = 8
FLAG_C2C2_MOBILITY = 16
FLAG_F_POPULATIONS = 32
FIELDS = {"C": 0, "V": 1, "P": 2, "F": 3, "MU": 4, "F_RAW": 5, "G_RAW": 6}
PRECISIONS = {"fp64": FP64, "fp32": FP32, "fp16s": FP16S}
BATCH_MODES = {"launch": 0, "graph": 1, "per_sim": 2}
STATUS = {0: "OK", -1: "EINVAL", -2: "ESINGULAR", -3: "EUNSTABLE", -4: "ENOMEM",
          -5: "EDEVICE", -6: "ENUMERIC", -7: "ENOTSUP"}


class NflbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class Config(ctypes.Structure):
    _fields_ = [
        ("lattice", ctypes.c_int),
        ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
        ("wall", ctypes.c_int * 3),
        ("ncomp", ctypes.c_int),
        ("implicit_comp", ctypes.c_int),
        ("sigma", ctypes.POINTER(ctypes.c_double)),
        ("width_D", ctypes.c_double),
        ("omega_stab", ctypes.c_double),
        ("tau", ctypes.POINTER(ctypes.c_double)),
        ("trt_magic", ctypes.c_double),
        ("tau_g", ctypes.POINTER(ctypes.c_double)),
        ("m", ctypes.c_double),
        ("body_force", ctypes.c_double * 3),
        ("precision", ctypes.c_int),
        ("flags", ctypes.c_int),
    ]


class Diag(ctypes.Structure):
    _fields_ = [
        ("mass", ctypes.c_double * MAX_COMP),
        ("momentum", ctypes.c_double * 3),
        ("max_abs_c", ctypes.c_double * MAX_COMP),
        ("min_c", ctypes.c_double * MAX_COMP),
        ("max_sum_dev", ctypes.c_double),
        ("vcm", ctypes.c_double * 3),
        ("vcm_component", ctypes.c_int),
        ("nan", ctypes.c_int),
    ]


_lib = None


def lib():
    """The loaded libnflbm.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2605_22214_amd.build`")
        # One HIP runtime per process: PyTorch for ROCm ships its own copy of
        # the HIP and HSA runtimes under the same library names.  Loaded first,
        # it is the one this library binds to; loaded after this library it
        # would start a second runtime that finds no GPU.  So torch, where
        # installed, is imported before the library is opened.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        P, I, D, LL = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
        DP = ctypes.POINTER(ctypes.c_double)
        sigs = {
            "nflbm_create": (I, [ctypes.POINTER(Config), ctypes.POINTER(P)]),
            "nflbm_destroy": (None, [P]),
            "nflbm_set_stream": (I, [P, P]),
            "nflbm_set_fields": (I, [P, DP, DP, DP]),
            "nflbm_step": (I, [P, LL]),
            "nflbm_synchronize": (I, [P]),
            "nflbm_set_nan_check": (I, [P, LL]),
            "nflbm_set_conc_launch": (I, [P, I, I]),
            "nflbm_set_solid": (I, [P, ctypes.c_void_p]),
            "nflbm_set_open_face": (I, [P, I, DP, DP]),
            "nflbm_set_outflow": (I, [P, I]),
            "nflbm_get_conc_launch": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I)]),
            "nflbm_step_timed": (I, [P, LL, DP, DP]),
            "nflbm_step_timed_kernels": (I, [P, LL, DP, DP]),
            "nflbm_get_field": (I, [P, I, DP]),
            "nflbm_state_bytes": (I, [P, ctypes.POINTER(ctypes.c_size_t)]),
            "nflbm_get_state": (I, [P, P]),
            "nflbm_set_state": (I, [P, P]),
            "nflbm_diagnostics": (I, [P, I, ctypes.POINTER(Diag)]),
            "nflbm_diagnostics_noalloc": (I, [P, I, ctypes.POINTER(Diag)]),
            "nflbm_coefficients": (I, [I, DP, D, DP, DP, DP, DP, DP]),
            "nflbm_bytes_per_node": (I, [P, DP]),
            "nflbm_set_launch": (I, [P, I, I]),
            "nflbm_get_launch": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
            "nflbm_last_error": (ctypes.c_char_p, [P]),
            "nflbm_abi_version": (I, []),
            "nflbm_autotune": (I, [P, ctypes.c_char_p]),
            "nflbm_storage_form": (I, [P]),
            "nflbm_f_storage_form": (I, [P]),
            "nflbm_device_bytes": (I, [ctypes.POINTER(Config), ctypes.POINTER(ctypes.c_size_t)]),
            "nflbm_bind_state": (I, [P, P, ctypes.c_size_t]),
            "nflbm_get_coeffs": (I, [P, DP, DP]),
            "nflbm_domain_size": (I, [P, DP]),
            "nflbm_batch_create": (I, [ctypes.POINTER(Config), I, ctypes.POINTER(P)]),
            "nflbm_batch_destroy": (None, [P]),
            "nflbm_batch_count": (I, [P]),
            "nflbm_batch_member": (P, [P, I]),
            "nflbm_batch_set_stream": (I, [P, P]),
            "nflbm_batch_set_fields": (I, [P, I, DP, DP, DP]),
            "nflbm_batch_get_field": (I, [P, I, I, DP]),
            "nflbm_batch_step": (I, [P, LL, I]),
            "nflbm_batch_step_timed": (I, [P, LL, I, DP]),
            "nflbm_batch_set_launch": (I, [P, I, I]),
            "nflbm_batch_get_launch": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I)]),
            "nflbm_batch_nodes": (I, [P, ctypes.POINTER(LL)]),
            "nflbm_batch_autotune": (I, [P, ctypes.c_char_p]),
            "nflbm_batch_last_error": (ctypes.c_char_p, [P]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def header_functions():
    """Names of the functions declared in include/nflbm.h."""
    with open(HEADER) as fh:
        text = fh.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nflbm_[a-z_0-9]+)\s*\(", text)))


def _dptr(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(code, handle=None):
    if code != 0:
        msg = lib().nflbm_last_error(handle)
        raise NflbmError(code, msg.decode() if msg else "")


def _bcheck(code, handle=None):
    if code != 0:
        msg = lib().nflbm_batch_last_error(handle)
        raise NflbmError(code, msg.decode() if msg else "")


class _Problem:
    """An nflbm_config together with the arrays it points into."""

    def __init__(self, lattice, shape, sigma, tau, *, walls=(False, False, False),
                 implicit=-1, D=4.0, omega_stab=0.0, trt_magic=0.0, tau_g=None, m=0.02,
                 body_force=(0.0, 0.0, 0.0), precision=FP64, flags=0):
        self.lattice = {"D2Q9": D2Q9, "D3Q19": D3Q19}.get(lattice, lattice)
        self.Q = 9 if self.lattice == D2Q9 else 19
        self.shape = tuple(int(s) for s in shape)
        nx, ny, nz = self.shape
        self.n = nx * ny * nz
        self.sigma = np.ascontiguousarray(sigma, dtype=np.float64)
        self.N = self.sigma.shape[0]
        self.tau = np.ascontiguousarray(np.broadcast_to(np.asarray(tau, float), (self.N,)))
        self.tau_g = None if tau_g is None else np.ascontiguousarray(
            np.broadcast_to(np.asarray(tau_g, float), (self.N,)))
        self.precision = PRECISIONS.get(precision, precision)
        cfg = Config()
        cfg.lattice = self.lattice
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        for a in range(3):
            cfg.wall[a] = int(bool(walls[a]))
        cfg.ncomp = self.N
        cfg.implicit_comp = -1 if implicit is None else int(implicit)
        cfg.sigma = _dptr(self.sigma)
        cfg.width_D = float(D)
        cfg.omega_stab = float(omega_stab)
        cfg.tau = _dptr(self.tau)
        cfg.trt_magic = float(trt_magic)
        cfg.tau_g = _dptr(self.tau_g) if self.tau_g is not None else None
        cfg.m = float(m)
        for a in range(3):
            cfg.body_force[a] = float(body_force[a])
        cfg.precision = int(self.precision)
        cfg.flags = int(flags)
        self.cfg = cfg

    @classmethod
    def from_workload(cls, w, precision=FP64, implicit=-1, flags=0):
        return cls(w["lattice"], w["shape"], w["sigma"], w["tau"], walls=w["walls"],
                   implicit=implicit, D=w["D"], omega_stab=w["omega_stab"],
                   trt_magic=w["trt_magic"], tau_g=w["tau_g"], m=w["m"],
                   body_force=w["body_force"], precision=precision, flags=flags)


def coefficients(sigma, D=4.0):
    """Host-side coefficient tables computed by the library (no GPU needed)."""
    sigma = np.ascontiguousarray(sigma, dtype=np.float64)
    N = sigma.shape[0]
    alpha = np.zeros((N, N))
    gamma = np.zeros(N)
    psi = np.zeros((N, N, N))
    xt = np.zeros((N, N, N))
    zt = np.zeros((N, N, N))
    _check(lib().nflbm_coefficients(N, _dptr(sigma), float(D), _dptr(alpha), _dptr(gamma),
                                    _dptr(psi), _dptr(xt), _dptr(zt)))
    return dict(alpha=alpha, gamma=gamma, psi=psi, X=xt, Z=zt)


class Simulation:
    """One lattice on the current HIP device (see include/nflbm.h)."""

    def __init__(self, lattice, shape, sigma, tau, **kw):
        self._adopt(_Problem(lattice, shape, sigma, tau, **kw))
        h = ctypes.c_void_p()
        _check(lib().nflbm_create(ctypes.byref(self._prob.cfg), ctypes.byref(h)))
        self._h = h
        self._owned = True

    def _adopt(self, prob):
        self._prob = prob
        self.lattice, self.Q, self.shape, self.n = prob.lattice, prob.Q, prob.shape, prob.n
        self.N, self.precision = prob.N, prob.precision

    @classmethod
    def _borrowed(cls, handle, prob):
        """A member of a Batch: the batch owns (and frees) the handle."""
        self = cls.__new__(cls)
        self._adopt(prob)
        self._h = ctypes.c_void_p(handle)
        self._owned = False
        return self

    @classmethod
    def from_workload(cls, w, precision=FP64, implicit=-1, flags=0):
        return cls(w["lattice"], w["shape"], w["sigma"], w["tau"], walls=w["walls"],
                   implicit=implicit, D=w["D"], omega_stab=w["omega_stab"],
                   trt_magic=w["trt_magic"], tau_g=w["tau_g"], m=w["m"],
                   body_force=w["body_force"], precision=precision, flags=flags)

    @property
    def grid(self):
        nx, ny, nz = self.shape
        return (nz, ny, nx)

    def _handle(self):
        if self._h is None:
            raise RuntimeError("simulation already closed")
        return self._h

    def set_stream(self, stream_ptr):
        _check(lib().nflbm_set_stream(self._handle(), ctypes.c_void_p(stream_ptr)), self._h)

    def set_fields(self, C, v=None, P=None):
        C = np.ascontiguousarray(np.asarray(C, dtype=np.float64).reshape(self.N, self.n))
        vv = None if v is None else np.ascontiguousarray(np.asarray(v, float).reshape(3, self.n))
        PP = None if P is None else np.ascontiguousarray(np.asarray(P, float).reshape(self.n))
        _check(lib().nflbm_set_fields(self._handle(), _dptr(C),
                                      _dptr(vv) if vv is not None else None,
                                      _dptr(PP) if PP is not None else None), self._h)

    def step(self, nsteps=1):
        _check(lib().nflbm_step(self._handle(), int(nsteps)), self._h)

    def synchronize(self):
        """Wait for the queued steps; raises NflbmError (ENUMERIC) if a
        checked step saw a NaN or Inf."""
        _check(lib().nflbm_synchronize(self._handle()), self._h)

    def set_nan_check(self, every):
        """Check for non-finite values on every `every`-th step (0: never)."""
        _check(lib().nflbm_set_nan_check(self._handle(), int(every)), self._h)

    def step_timed(self, nsteps, per_update=False):
        """Device milliseconds for nsteps (HIP events on the sim's stream);
        with per_update also the summed duration of the update launches."""
        ms = ctypes.c_double()
        mu = ctypes.c_double()
        _check(lib().nflbm_step_timed(self._handle(), int(nsteps), ctypes.byref(ms),
                                      ctypes.byref(mu) if per_update else None), self._h)
        return (ms.value, mu.value) if per_update else ms.value

    def step_timed_kernels(self, nsteps):
        """Summed device milliseconds of the reconstruction and of the update
        launches over nsteps (HIP events around each launch)."""
        mc = ctypes.c_double()
        mu = ctypes.c_double()
        _check(lib().nflbm_step_timed_kernels(self._handle(), int(nsteps), ctypes.byref(mc),
                                              ctypes.byref(mu)), self._h)
        return mc.value, mu.value

    def get_field(self, name):
        fid = FIELDS[name]
        rows = {"C": self.N, "V": 3, "P": 1, "F": 3, "MU": self.N,
                "F_RAW": self.Q - 1, "G_RAW": self.N * self.Q}[name]
        out = np.empty(rows * self.n, dtype=np.float64)
        _check(lib().nflbm_get_field(self._handle(), fid, _dptr(out)), self._h)
        if name == "G_RAW":
            return out.reshape((self.N, self.Q) + self.grid)
        if name == "P":
            return out.reshape(self.grid)
        return out.reshape((rows,) + self.grid)

    def state_bytes(self):
        b = ctypes.c_size_t()
        _check(lib().nflbm_state_bytes(self._handle(), ctypes.byref(b)), self._h)
        return b.value

    def get_state(self):
        buf = np.empty(self.state_bytes(), dtype=np.uint8)
        _check(lib().nflbm_get_state(self._handle(), buf.ctypes.data_as(ctypes.c_void_p)), self._h)
        return buf

    def set_state(self, buf):
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        if buf.size != self.state_bytes():
            raise ValueError("state size mismatch")
        _check(lib().nflbm_set_state(self._handle(), buf.ctypes.data_as(ctypes.c_void_p)), self._h)

    def diagnostics(self, vcm_component=0, check=True):
        d = Diag()
        code = lib().nflbm_diagnostics(self._handle(), int(vcm_component), ctypes.byref(d))
        return self._diag_dict(d, code, check)

    def diagnostics_noalloc(self, vcm_component=0, check=True):
        """nflbm_diagnostics_noalloc: the same diagnostics without any device
        allocation (the library's fixed array holds the partial sums)."""
        d = Diag()
        code = lib().nflbm_diagnostics_noalloc(self._handle(), int(vcm_component), ctypes.byref(d))
        return self._diag_dict(d, code, check)

    def _diag_dict(self, d, code, check):
        if check:
            _check(code, self._h)
        N = self.N
        return {"mass": list(d.mass[:N]), "momentum": list(d.momentum),
                "max_abs_c": list(d.max_abs_c[:N]), "min_c": list(d.min_c[:N]),
                "max_sum_dev": d.max_sum_dev, "vcm": list(d.vcm), "nan": d.nan,
                "status": code}

    def set_launch(self, tx_log2=0, zchunk=0):
        _check(lib().nflbm_set_launch(self._handle(), int(tx_log2), int(zchunk)), self._h)

    def get_launch(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(lib().nflbm_get_launch(self._handle(), ctypes.byref(a), ctypes.byref(b),
                                      ctypes.byref(c)), self._h)
        return a.value, b.value, c.value

    def set_solid(self, solid):
        """Solid nodes (bool or 0/1 array in [nz][ny][nx] order, or None to
        remove them); call before set_fields."""
        if solid is None:
            _check(lib().nflbm_set_solid(self._handle(), None), self._h)
            return
        m = np.ascontiguousarray(np.asarray(solid).reshape(-1) != 0, dtype=np.uint8)
        if m.size != int(np.prod(self.shape)):
            raise ValueError("solid mask must have one entry per node")
        _check(lib().nflbm_set_solid(self._handle(), m.ctypes.data), self._h)

    def set_open_face(self, face, v_b=None, C_b=None):
        """Open face 0..5 (x-, x+, y-, y+, z-, z+) with velocity v_b and
        concentrations C_b (user order), or a wall again with None."""
        if v_b is None:
            _check(lib().nflbm_set_open_face(self._handle(), int(face), None, None), self._h)
            return
        v = np.ascontiguousarray(v_b, dtype=np.float64).reshape(3)
        c = np.ascontiguousarray(C_b, dtype=np.float64).reshape(self.N)
        _check(lib().nflbm_set_open_face(self._handle(), int(face), _dptr(v), _dptr(c)), self._h)

    def set_outflow(self, face):
        """Convective outflow on face 0..5 (x-, x+, y-, y+, z-, z+), or None
        to remove it."""
        _check(lib().nflbm_set_outflow(self._handle(), -1 if face is None else int(face)), self._h)

    def set_conc_launch(self, tx_log2=0, zchunk=0):
        _check(lib().nflbm_set_conc_launch(self._handle(), int(tx_log2), int(zchunk)), self._h)

    def get_conc_launch(self):
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().nflbm_get_conc_launch(self._handle(), ctypes.byref(a), ctypes.byref(b)), self._h)
        return a.value, b.value

    def bytes_per_node(self):
        b = ctypes.c_double()
        _check(lib().nflbm_bytes_per_node(self._handle(), ctypes.byref(b)), self._h)
        return b.value

    @staticmethod
    def device_bytes(lattice, shape, sigma, tau, **kw):
        """Device bytes the state of such a simulation occupies (no GPU use)."""
        prob = _Problem(lattice, shape, sigma, tau, **kw)
        b = ctypes.c_size_t()
        _check(lib().nflbm_device_bytes(ctypes.byref(prob.cfg), ctypes.byref(b)))
        return b.value

    def bind_state(self, dev_ptr, nbytes):
        """Keep the state in caller memory (e.g. tensor.data_ptr()); the caller
        keeps that memory alive while the simulation exists."""
        _check(lib().nflbm_bind_state(self._handle(), ctypes.c_void_p(dev_ptr), ctypes.c_size_t(nbytes)),
               self._h)

    def get_coeffs(self):
        a = np.zeros((self.N, self.N))
        g = np.zeros(self.N)
        _check(lib().nflbm_get_coeffs(self._handle(), _dptr(a), _dptr(g)), self._h)
        return a, g

    def domain_size(self):
        """L_i of Eq. L for every component (lattice units)."""
        out = np.zeros(self.N)
        _check(lib().nflbm_domain_size(self._handle(), _dptr(out)), self._h)
        return out

    def storage_form(self):
        """'moments' (g kept as C, mu~, v per node; every tau_g = 1) or 'populations'."""
        r = lib().nflbm_storage_form(self._handle())
        if r < 0:
            _check(r, self._h)
        return "moments" if r == 1 else "populations"

    def f_storage_form(self):
        """'records' (f kept as (fA, F) per node; every omega = 1) or 'populations'."""
        r = lib().nflbm_f_storage_form(self._handle())
        if r < 0:
            _check(r, self._h)
        return "records" if r == 1 else "populations"

    def autotune(self, cache_path=None):
        """Time the launch shapes and keep the fastest (state unchanged)."""
        _check(lib().nflbm_autotune(self._handle(), None if cache_path is None
                                    else os.fsencode(cache_path)), self._h)
        return self.get_launch() + self.get_conc_launch()

    def close(self):
        if getattr(self, "_h", None) is not None:
            if getattr(self, "_owned", True):
                lib().nflbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


class Batch:
    """Independent simulations of one lattice, N and precision advanced
    together (see include/nflbm.h).  members: _Problem-style keyword dicts
    (``lattice, shape, sigma, tau`` plus the Simulation keywords) or workload
    dicts with ``from_workloads``."""

    def __init__(self, problems):
        probs = [p if isinstance(p, _Problem) else _Problem(**p) for p in problems]
        if not probs:
            raise ValueError("a batch needs at least one member")
        arr = (Config * len(probs))(*[p.cfg for p in probs])
        h = ctypes.c_void_p()
        _bcheck(lib().nflbm_batch_create(arr, len(probs), ctypes.byref(h)))
        self._h = h
        self._probs = probs
        self.members = [Simulation._borrowed(lib().nflbm_batch_member(h, i), p)
                        for i, p in enumerate(probs)]

    @classmethod
    def from_workloads(cls, ws, precision=FP64, implicit=-1, flags=0):
        return cls([_Problem.from_workload(w, precision=precision, implicit=implicit, flags=flags)
                    for w in ws])

    def _handle(self):
        if self._h is None:
            raise RuntimeError("batch already closed")
        return self._h

    def __len__(self):
        return len(self.members)

    def nodes(self):
        n = ctypes.c_longlong()
        _bcheck(lib().nflbm_batch_nodes(self._handle(), ctypes.byref(n)), self._h)
        return n.value

    def set_stream(self, stream_ptr):
        _bcheck(lib().nflbm_batch_set_stream(self._handle(), ctypes.c_void_p(stream_ptr)), self._h)

    def set_fields(self, idx, C, v=None, P=None):
        """nflbm_batch_set_fields of member idx (also clears the batch's NaN flag)."""
        m = self.members[idx]
        C = np.ascontiguousarray(C, dtype=np.float64).reshape(m.N, -1)
        vv = None if v is None else np.ascontiguousarray(v, dtype=np.float64).reshape(3, -1)
        PP = None if P is None else np.ascontiguousarray(P, dtype=np.float64).reshape(-1)
        _bcheck(lib().nflbm_batch_set_fields(self._handle(), int(idx), _dptr(C),
                                             _dptr(vv) if vv is not None else None,
                                             _dptr(PP) if PP is not None else None), self._h)

    def step(self, nsteps=1, mode="graph"):
        _bcheck(lib().nflbm_batch_step(self._handle(), int(nsteps), BATCH_MODES[mode]), self._h)

    def step_timed(self, nsteps, mode="graph"):
        ms = ctypes.c_double()
        _bcheck(lib().nflbm_batch_step_timed(self._handle(), int(nsteps), BATCH_MODES[mode],
                                             ctypes.byref(ms)), self._h)
        return ms.value

    def set_launch(self, tx_log2=0, graph_steps=0):
        _bcheck(lib().nflbm_batch_set_launch(self._handle(), int(tx_log2), int(graph_steps)), self._h)

    def get_launch(self):
        a, b, c = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _bcheck(lib().nflbm_batch_get_launch(self._handle(), ctypes.byref(a), ctypes.byref(b),
                                             ctypes.byref(c)), self._h)
        return a.value, b.value, c.value

    def autotune(self, cache_path=None):
        _bcheck(lib().nflbm_batch_autotune(self._handle(), None if cache_path is None
                                           else os.fsencode(cache_path)), self._h)
        return self.get_launch()

    def close(self):
        if getattr(self, "_h", None) is not None:
            for m in self.members:
                m._h = None
            lib().nflbm_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
