"""MI355X pseudo-spectral stochastic-PDE stepper (cuPSS method, arXiv 2405.02410).

Thin ctypes binding over the C interface in include/pss.h.  Every step of the
hot path runs in the HIP kernels of libpss.so; this module only marshals
arguments.  Device arrays may be passed as torch tensors (their data pointer
is used); host arrays as numpy arrays.

Terms follow the paper's form (eq:basereal): each term adds
op(q) * prod_j field_j^p_j to d/dt of its target.  An operator is a list of
monomials coef * (q^2)^q2 * |q|^-invq * prod_i (i q_i)^iq_i (Sec. "Reserved
keywords").  Implicit terms (treated by the 1/(1 - dt L) factor of
eq:timeupdate) must be linear in their own field.
"""

import ctypes
import os
from collections import namedtuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# PSS_LIB names another build of the same library (the host-sanitizer build
# that the CPU interface tests run under); by default the in-tree libpss.so
_LIB_PATH = os.environ.get("PSS_LIB") or os.path.join(_HERE, "libpss.so")

PSS_OK = 0
ERRORS = {
    -1: "PSS_E_INVAL",
    -2: "PSS_E_UNSUPPORTED",
    -3: "PSS_E_NOMEM",
    -4: "PSS_E_HIP",
    -5: "PSS_E_STATE",
    -6: "PSS_E_UNSTABLE",
    -7: "PSS_E_NONFINITE",
}
DEALIAS_TWO_THIRDS, DEALIAS_PAPER_ORDER, DEALIAS_NONE = 0, 1, 2
SHAPE_RADIAL, SHAPE_PER_AXIS = 0, 1
KERNEL_UPDATE, KERNEL_X = 0, 1


class PssError(RuntimeError):
    def __init__(self, code, msg):
        self.code = code
        self.name = ERRORS.get(code, str(code))
        super().__init__(f"{self.name}: {msg}")


class _QMono(ctypes.Structure):
    _fields_ = [("coef", ctypes.c_double), ("q2_pow", ctypes.c_int32),
                ("invq_pow", ctypes.c_int32), ("iq_pow", ctypes.c_int32 * 3)]


Mono = namedtuple("Mono", ["coef", "q2", "invq", "iq"], defaults=(0, 0, (0, 0, 0)))

_lib = None

_SIGS = {
    "pss_lattice_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32, ctypes.POINTER(ctypes.c_int64),
                           ctypes.POINTER(ctypes.c_double), ctypes.c_double],
    "pss_lattice_destroy": [ctypes.c_void_p],
    "pss_field_declare": [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)],
    "pss_term_add": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(_QMono), ctypes.c_int32,
                     ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                     ctypes.POINTER(ctypes.c_int32)],
    "pss_term_set_coef": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_double],
    "pss_frame_set": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64],
    "pss_param_set": [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_double],
    "pss_param_get": [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double)],
    "pss_field_find": [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
    "pss_equation_add": [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                         ctypes.POINTER(ctypes.c_int32)],
    "pss_noise_expr": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_char_p],
    "pss_term_info": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                      ctypes.POINTER(_QMono), ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
    "pss_term_count": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)],
    "pss_noise_set": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(_QMono), ctypes.c_int32],
    "pss_seed_set": [ctypes.c_void_p, ctypes.c_uint64],
    "pss_dealias_set": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32],
    "pss_stream_set": [ctypes.c_void_p, ctypes.c_void_p],
    "pss_validate": [ctypes.c_void_p],
    "pss_field_upload": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32],
    "pss_field_init_uniform": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_double],
    "pss_field_download": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32],
    "pss_spectrum_download": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32],
    "pss_step": [ctypes.c_void_p, ctypes.c_int64],
    "pss_step_index": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)],
    "pss_sync": [ctypes.c_void_p],
    "pss_state_size": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_size_t)],
    "pss_field_bind": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_size_t],
    "pss_field_state_bytes": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)],
    "pss_state_changed": [ctypes.c_void_p],
    "pss_state_save": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "pss_state_load": [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t],
    "pss_mass": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
    "pss_structure_factor": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32],
    "pss_util_philox": [ctypes.c_uint32] * 6 + [ctypes.c_int64, ctypes.c_void_p],
    "pss_time_kernel": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                        ctypes.POINTER(ctypes.c_char_p)],
    "pss_kernel_bytes": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
    "pss_kernels_per_step": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32)],
    "pss_tuning_set": [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64],
    "pss_tuning_get": [ctypes.c_void_p, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int64)],
    "pss_autotune": [ctypes.c_void_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_double)],
    "pss_adjoint_model_b": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                            ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double),
                            ctypes.c_void_p, ctypes.c_int32],
    "pss_adjoint_model_b_forward": [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_void_p)],
    "pss_adjoint_model_b_backward": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double), ctypes.c_void_p,
                                     ctypes.c_int32],
    "pss_tape_destroy": [ctypes.c_void_p],
    "pss_step_prepare": [ctypes.c_void_p, ctypes.c_int64],
    "pss_structure_factor_noalloc": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_int32],
    "pss_batch_create": [ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p), ctypes.c_int32,
                         ctypes.POINTER(ctypes.c_uint64)],
    "pss_batch_destroy": [ctypes.c_void_p],
    "pss_batch_step": [ctypes.c_void_p, ctypes.c_int64],
    "pss_batch_sync": [ctypes.c_void_p],
    "pss_batch_info": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
    "pss_batch_launches": [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                           ctypes.POINTER(ctypes.c_int32)],
    "pss_batch_time_kernel": [ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                              ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)],
}


def lib():
    """Load libpss.so (built by paper_2405_02410_amd.build); raise if missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with "
                              "`python -m paper_2405_02410_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(_LIB_PATH)
        for name, argt in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = argt
            fn.restype = ctypes.c_int32
        L.pss_last_error.argtypes = []
        L.pss_last_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(code):
    if code != PSS_OK:
        raise PssError(code, lib().pss_last_error().decode())


def _monos(op):
    op = [m if isinstance(m, Mono) else Mono(*m) for m in op]
    arr = (_QMono * len(op))()
    for i, m in enumerate(op):
        iq = tuple(m.iq) + (0,) * (3 - len(m.iq))
        arr[i].coef = float(m.coef)
        arr[i].q2_pow = int(m.q2)
        arr[i].invq_pow = int(m.invq)
        for k in range(3):
            arr[i].iq_pow[k] = int(iq[k])
    return arr, len(op)


def _ptr(a):
    """(address, on_device) of a torch tensor or numpy array of float32."""
    if hasattr(a, "data_ptr"):
        if a.dtype.__str__() != "torch.float32" or not a.is_contiguous():
            raise TypeError("torch tensors must be contiguous float32")
        return a.data_ptr(), 1 if a.is_cuda else 0
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a.ctypes.data, 0


class Lattice:
    """A periodic 1D, 2D or 3D lattice with fields, terms and noise (one context)."""

    def __init__(self, n, dx=None, dt=0.01, seed=0, dealias=DEALIAS_TWO_THIRDS, shape=SHAPE_RADIAL):
        n = tuple(int(v) for v in n)
        self.ndim = len(n)
        if self.ndim not in (1, 2, 3):
            raise PssError(-2, f"ndim must be 1, 2 or 3 (got {self.ndim})")
        dx = tuple(float(v) for v in (dx if dx is not None else (1.0,) * self.ndim))
        n3 = (ctypes.c_int64 * 3)(*(n + (1,) * (3 - self.ndim)))
        d3 = (ctypes.c_double * 3)(*(dx + (1.0,) * (3 - self.ndim)))
        h = ctypes.c_void_p()
        _check(lib().pss_lattice_create(ctypes.byref(h), self.ndim, n3, d3, float(dt)))
        self._h = h
        self.n = n
        self.dx = dx
        self.dt = float(dt)
        self.shape = tuple(reversed(n))  # numpy order (z, y, x)
        self.sites = int(np.prod(n))
        self.names = []
        self._bound = []  # tensors that hold field states (kept alive with the lattice)
        _check(lib().pss_seed_set(self._h, int(seed) & 0xFFFFFFFFFFFFFFFF))
        _check(lib().pss_dealias_set(self._h, int(dealias), int(shape)))

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().pss_lattice_destroy(self._h))  # fails while a batch holds it
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- model ---------------------------------------------------------
    def field(self, name, dynamic=True):
        fid = ctypes.c_int32()
        _check(lib().pss_field_declare(self._h, name.encode(), int(dynamic), ctypes.byref(fid)))
        self.names.append(name)
        return fid.value

    def term(self, target, op, factors, implicit=False):
        arr, nm = _monos(op)
        ff = (ctypes.c_int32 * len(factors))(*[int(f) for f, _ in factors])
        fp = (ctypes.c_int32 * len(factors))(*[int(p) for _, p in factors])
        tid = ctypes.c_int32()
        _check(lib().pss_term_add(self._h, int(target), int(implicit), arr, nm, ff, fp, len(factors),
                                  ctypes.byref(tid)))
        return tid.value

    def set_coef(self, term, mono, coef):
        _check(lib().pss_term_set_coef(self._h, int(term), int(mono), float(coef)))

    def noise(self, field, op):
        arr, nm = _monos(op)
        _check(lib().pss_noise_set(self._h, int(field), arr, nm))

    # -- equation front end (Sec. "Writing models") -------------------
    def param(self, name, value):
        """Named parameter for equation strings (addParameter)."""
        _check(lib().pss_param_set(self._h, name.encode(), float(value)))

    def field_id(self, name):
        """Declaration index of the field called `name`."""
        fid = ctypes.c_int32()
        _check(lib().pss_field_find(self._h, name.encode(), ctypes.byref(fid), None))
        return fid.value

    def equation(self, text):
        """Add the terms of an equation string such as
        "dt phi + (a*q^2 + k*q^4)*phi = -b*q^2*phi^3"; returns the ids of the
        terms added."""
        first, n = ctypes.c_int32(), ctypes.c_int32()
        _check(lib().pss_equation_add(self._h, text.encode(), ctypes.byref(first), ctypes.byref(n)))
        return list(range(first.value, first.value + n.value))

    def noise_expr(self, field, expr):
        """Noise of `field` from a prefactor string such as "D*q^2" (addNoise)."""
        _check(lib().pss_noise_expr(self._h, int(field), expr.encode()))

    def terms(self):
        """Every term as added: (target, implicit, [Mono], [(field, power)])."""
        n = ctypes.c_int32()
        _check(lib().pss_term_count(self._h, ctypes.byref(n)))
        out = []
        for t in range(n.value):
            tgt, imp, nm, nf = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
            ops = (_QMono * 8)()
            ff = (ctypes.c_int32 * 4)()
            fp = (ctypes.c_int32 * 4)()
            _check(lib().pss_term_info(self._h, t, ctypes.byref(tgt), ctypes.byref(imp), ops, ctypes.byref(nm),
                                       ff, fp, ctypes.byref(nf)))
            monos = [Mono(ops[i].coef, ops[i].q2_pow, ops[i].invq_pow, tuple(ops[i].iq_pow)) for i in range(nm.value)]
            out.append((tgt.value, bool(imp.value), monos, [(ff[i], fp[i]) for i in range(nf.value)]))
        return out

    def frame(self, field, sites, values):
        """Hold `field` at `values` on the linear real-space sites `sites`
        after every step (a boundary frame); empty arrays remove it."""
        st = np.ascontiguousarray(np.asarray(sites, dtype=np.int64).reshape(-1))
        vs = np.ascontiguousarray(np.asarray(values, dtype=np.float32).reshape(-1))
        if st.shape != vs.shape:
            raise PssError(-1, "frame sites and values differ in length")
        _check(lib().pss_frame_set(self._h, int(field), st.ctypes.data_as(ctypes.c_void_p),
                                   vs.ctypes.data_as(ctypes.c_void_p), int(st.size)))

    def seed(self, seed):
        _check(lib().pss_seed_set(self._h, int(seed) & 0xFFFFFFFFFFFFFFFF))

    def stream(self, hip_stream):
        """Run on a hipStream_t given as an integer handle (torch: stream.cuda_stream)."""
        _check(lib().pss_stream_set(self._h, ctypes.c_void_p(int(hip_stream) if hip_stream else 0)))

    def tune(self, **kw):
        """Force launch-geometry values (tc, to, tz, rb, pu, px, py) before the plan is built."""
        for k, v in kw.items():
            _check(lib().pss_tuning_set(self._h, k.encode(), int(v)))

    def autotune(self, reps=30):
        """Time candidate launch geometries and keep the fastest (pss_autotune);
        returns the summed kernel time of one step in microseconds."""
        us = ctypes.c_double()
        _check(lib().pss_autotune(self._h, int(reps), ctypes.byref(us)))
        return us.value

    def geometry(self):
        out = {}
        for k in ("tc", "to", "tz", "rb", "pu", "px", "py"):
            v = ctypes.c_int64()
            _check(lib().pss_tuning_get(self._h, k.encode(), ctypes.byref(v)))
            out[k] = v.value
        return out

    def validate(self):
        _check(lib().pss_validate(self._h))

    # -- state ---------------------------------------------------------
    def upload(self, field, values):
        if hasattr(values, "data_ptr"):
            if values.numel() != self.sites:
                raise ValueError("wrong number of sites")
            p, dev = _ptr(values)
            _check(lib().pss_field_upload(self._h, int(field), ctypes.c_void_p(p), dev))
        else:
            a = np.ascontiguousarray(values, dtype=np.float32).reshape(-1)
            if a.size != self.sites:
                raise ValueError("wrong number of sites")
            _check(lib().pss_field_upload(self._h, int(field), a.ctypes.data_as(ctypes.c_void_p), 0))

    def init_uniform(self, field, lo=-0.1, hi=0.1):
        _check(lib().pss_field_init_uniform(self._h, int(field), float(lo), float(hi)))

    def download(self, field, out=None):
        """Real-space field as a numpy array (z, y, x), or into a float32 torch tensor."""
        if out is not None and hasattr(out, "data_ptr"):
            p, dev = _ptr(out)
            _check(lib().pss_field_download(self._h, int(field), ctypes.c_void_p(p), dev))
            return out
        a = np.empty(self.shape, dtype=np.float32)
        _check(lib().pss_field_download(self._h, int(field), a.ctypes.data_as(ctypes.c_void_p), 0))
        return a

    def spectrum(self, field):
        """Half spectrum phi_hat(kx = 0..Nx/2) as complex64 array (z, y, kx)."""
        nh = self.n[0] // 2 + 1
        a = np.empty(self.shape[:-1] + (nh, 2), dtype=np.float32)
        _check(lib().pss_spectrum_download(self._h, int(field), a.ctypes.data_as(ctypes.c_void_p), 0))
        return a[..., 0] + 1j * a[..., 1]

    def state_bytes(self, field):
        """Bytes of the field's Fourier state (pss_field_state_bytes)."""
        v = ctypes.c_size_t()
        _check(lib().pss_field_state_bytes(self._h, int(field), ctypes.byref(v)))
        return v.value

    def bind(self, field, tensor):
        """Let a contiguous torch CUDA tensor of at least state_bytes(field)
        bytes hold the field's Fourier state (pss_field_bind); before the first
        call that builds the plan.  The lattice keeps a reference to it."""
        if not getattr(tensor, "is_cuda", False) or not tensor.is_contiguous():
            raise ValueError("bind takes a contiguous CUDA tensor")
        nbytes = tensor.numel() * tensor.element_size()
        _check(lib().pss_field_bind(self._h, int(field), ctypes.c_void_p(tensor.data_ptr()), nbytes))
        self._bound.append(tensor)

    def state_changed(self):
        """After writing a bound state tensor directly (pss_state_changed)."""
        _check(lib().pss_state_changed(self._h))

    def step(self, n=1):
        _check(lib().pss_step(self._h, int(n)))

    def prepare(self, n):
        """Build the plan and the step graphs that step(n) replays, without stepping."""
        _check(lib().pss_step_prepare(self._h, int(n)))

    def sync(self):
        _check(lib().pss_sync(self._h))

    @property
    def step_index(self):
        v = ctypes.c_int64()
        _check(lib().pss_step_index(self._h, ctypes.byref(v)))
        return v.value

    def save(self):
        n = ctypes.c_size_t()
        _check(lib().pss_state_size(self._h, ctypes.byref(n)))
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().pss_state_save(self._h, buf, n.value))
        return buf.raw

    def load(self, blob):
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        _check(lib().pss_state_load(self._h, buf, len(blob)))

    # -- reductions ----------------------------------------------------
    def mass(self, field):
        v = ctypes.c_double()
        _check(lib().pss_mass(self._h, int(field), ctypes.byref(v)))
        return v.value

    def structure_factor_noalloc(self, field):
        """structure_factor through the allocation-free entry point (the plan
        must be built)."""
        ns = min(n for n in self.n) // 2 - 1
        S = np.zeros(ns, dtype=np.float64)
        cnt = np.zeros(ns, dtype=np.int64)
        _check(lib().pss_structure_factor_noalloc(self._h, int(field), S.ctypes.data_as(ctypes.c_void_p),
                                                  cnt.ctypes.data_as(ctypes.c_void_p), ns))
        return S, cnt

    def structure_factor(self, field):
        ns = min(n for n in self.n) // 2 - 1
        S = np.zeros(ns, dtype=np.float64)
        cnt = np.zeros(ns, dtype=np.int64)
        _check(lib().pss_structure_factor(self._h, int(field), S.ctypes.data_as(ctypes.c_void_p),
                                          cnt.ctypes.data_as(ctypes.c_void_p), ns))
        return S, cnt

    # -- measurement helpers -------------------------------------------
    def time_kernel(self, which, reps):
        ms = ctypes.c_double()
        name = ctypes.c_char_p()
        _check(lib().pss_time_kernel(self._h, int(which), int(reps), ctypes.byref(ms), ctypes.byref(name)))
        return ms.value, name.value.decode()

    def kernel_bytes(self, which):
        b = ctypes.c_double()
        _check(lib().pss_kernel_bytes(self._h, int(which), ctypes.byref(b)))
        return b.value

    def adjoint_model_b(self, nsteps, S_target, ckpt_every=45, grad_phi0=True):
        """(loss, dL/d(a, b, k, D), dL/dphi_0 or None) of the structure-factor
        loss after nsteps Model B steps from the current state (pss_adjoint_model_b).
        Leaves the lattice at the end of the forward run."""
        S = np.ascontiguousarray(S_target, dtype=np.float64)
        loss = ctypes.c_double()
        grad = (ctypes.c_double * 4)()
        out = np.empty(self.shape, dtype=np.float32) if grad_phi0 else None
        _check(lib().pss_adjoint_model_b(self._h, int(nsteps), int(ckpt_every),
                                         S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(S.size),
                                         ctypes.byref(loss), grad,
                                         None if out is None else out.ctypes.data, 0))
        return loss.value, np.array(list(grad)), out

    def adjoint_forward(self, nsteps, S_target, ckpt_every=45):
        """Checkpointed forward phase of the Model B adjoint
        (pss_adjoint_model_b_forward): (loss, Tape)."""
        S = np.ascontiguousarray(S_target, dtype=np.float64)
        loss = ctypes.c_double()
        h = ctypes.c_void_p()
        _check(lib().pss_adjoint_model_b_forward(self._h, int(nsteps), int(ckpt_every),
                                                 S.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(S.size),
                                                 ctypes.byref(loss), ctypes.byref(h)))
        return loss.value, Tape(h, self)

    def kernels_per_step(self):
        v = ctypes.c_int32()
        _check(lib().pss_kernels_per_step(self._h, ctypes.byref(v)))
        return v.value


class Tape:
    """Recorded forward run of the Model B adjoint (pss_tape); backward() runs
    the reverse sweep once.  close() (or garbage collection) frees it."""

    def __init__(self, handle, lattice):
        self._h = handle
        self.lattice = lattice  # kept alive while the tape exists

    def backward(self, grad_phi0=None):
        """dL/d(a, b, k, D) as a numpy array; dL/dphi_0 into grad_phi0 (a float32
        torch tensor on the device, or a numpy array) when given."""
        grad = (ctypes.c_double * 4)()
        if grad_phi0 is None:
            _check(lib().pss_adjoint_model_b_backward(self._h, grad, None, 0))
        elif hasattr(grad_phi0, "data_ptr"):
            if grad_phi0.numel() != self.lattice.sites:
                raise ValueError("wrong number of sites")
            p, dev = _ptr(grad_phi0)
            _check(lib().pss_adjoint_model_b_backward(self._h, grad, ctypes.c_void_p(p), dev))
        else:
            if grad_phi0.size != self.lattice.sites or grad_phi0.dtype != np.float32 or \
                    not grad_phi0.flags.c_contiguous:
                raise ValueError("grad_phi0 must be a contiguous float32 array of every site")
            _check(lib().pss_adjoint_model_b_backward(self._h, grad, grad_phi0.ctypes.data, 0))
        return np.array(list(grad))

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().pss_tape_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Independent 2D lattices advanced together (pss_batch_*): one fused
    update and one fused x launch per step for the classes that fit them, one
    of each per step for any other size class.  Holds references to its lattices;
    close() (or garbage collection) frees the batch, not the lattices."""

    def __init__(self, lattices, seeds=None):
        self.lattices = list(lattices)
        n = len(self.lattices)
        hs = (ctypes.c_void_p * max(n, 1))(*[l._h for l in self.lattices])
        sd = None if seeds is None else (ctypes.c_uint64 * n)(*[int(v) for v in seeds])
        h = ctypes.c_void_p()
        _check(lib().pss_batch_create(ctypes.byref(h), hs, n, sd))
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().pss_batch_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, nsteps=1):
        _check(lib().pss_batch_step(self._h, int(nsteps)))

    def sync(self):
        _check(lib().pss_batch_sync(self._h))

    def classes(self):
        """(number of size classes, class of each member)."""
        nc = ctypes.c_int32()
        of = (ctypes.c_int32 * len(self.lattices))()
        _check(lib().pss_batch_info(self._h, ctypes.byref(nc), of))
        return nc.value, list(of)

    def launches(self):
        """(kernel launches per step outside the LDS-resident classes, classes
        in the fused launches, LDS-resident classes)."""
        per, fused, res = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(lib().pss_batch_launches(self._h, ctypes.byref(per), ctypes.byref(fused), ctypes.byref(res)))
        return per.value, fused.value, res.value

    def time_kernel(self, cls, which=KERNEL_UPDATE, reps=100):
        """(ms per launch, algorithmic bytes per launch) of one class's kernel,
        of the fused launch of that phase for cls = -1, or (ms, HBM bytes) per
        step of one launch of `reps` steps of the LDS-resident classes for
        cls = -2."""
        ms, b = ctypes.c_double(), ctypes.c_double()
        _check(lib().pss_batch_time_kernel(self._h, int(cls), int(which), int(reps), ctypes.byref(ms),
                                           ctypes.byref(b)))
        return ms.value, b.value


def philox(counter0, c1, c2, c3, k0, k1, count, out):
    """Philox4x32-10 words for counters (counter0 + i, c1, c2, c3) into a device uint32 tensor."""
    if not hasattr(out, "data_ptr") or not out.is_cuda or out.numel() < 4 * count:
        raise TypeError("out must be a device tensor with 4*count 32-bit elements")
    _check(lib().pss_util_philox(counter0, c1, c2, c3, k0, k1, int(count), ctypes.c_void_p(out.data_ptr())))


def model_b(lat, a=-1.0, b=1.0, k=1.0, D=0.01):
    """Model B (Cahn-Hilliard), Sec. "Example":
    d/dt phi = -q^2 (a + k q^2) phi - b q^2 F[phi^3] + conserved noise D q^2.
    Returns the field id and the term ids (implicit, cubic)."""
    f = lat.field("phi")
    t_imp = lat.term(f, [Mono(-a, q2=1), Mono(-k, q2=2)], [(f, 1)], implicit=True)
    t_nl = lat.term(f, [Mono(-b, q2=1)], [(f, 3)])
    if D:
        lat.noise(f, [Mono(D, q2=1)])
    return f, (t_imp, t_nl)


def kpz(lat, sigma=1.0, lam=1.0, D=0.01):
    """KPZ interface growth, Sec. "What cuPSS calculates":
    d/dt phi = sigma lap phi + lam (grad phi)^2 + sqrt(2 D) eta, written with one
    intermediate field per axis, g_i = d_i phi (i q_i phi), and explicit terms
    lam g_i^2.  Returns the field id of phi and the ids of the gradient fields."""
    f = lat.field("phi")
    lat.term(f, [Mono(-sigma, q2=1)], [(f, 1)], implicit=True)
    grads = []
    for i in range(lat.ndim):
        iq = [0, 0, 0]
        iq[i] = 1
        g = lat.field("d%s_phi" % "xyz"[i], dynamic=False)
        lat.term(g, [Mono(1.0, iq=tuple(iq))], [(f, 1)])
        lat.term(f, [Mono(lam)], [(g, 2)])
        grads.append(g)
    if D:
        lat.noise(f, [Mono(D)])
    return f, grads


def model_h(lat, a=-1.0, b=1.0, k=1.0, M=1.0, eta=1.0, D=0.0):
    """Model H in 2D or 3D (the paper's second benchmark, Sec. "Benchmarking"):
    a conserved order parameter advected by an incompressible viscous flow
    that its interfaces drive,
        d/dt phi = -v.grad phi + M lap mu,   mu = a phi + b phi^3 - k lap phi,
        d/dt v = eta lap v - grad p - phi grad mu,   div v = 0,
    with conserved noise D q^2 on phi.  The pressure is the projection
    P_ij = delta_ij + (i q_i)(i q_j)/q^2 folded into the operators of the
    force terms, the force written as -k d_j(g_i g_j), g = grad phi (it
    differs from -phi grad mu by a gradient, which the projection removes).
    Returns (phi, v_x, v_y[, v_z]) and the ids of the gradient fields."""
    nd = lat.ndim
    if nd not in (2, 3):
        raise ValueError("model_h is two- or three-dimensional")
    phi = lat.field("phi")
    v = [lat.field("v" + "xyz"[i]) for i in range(nd)]
    g = [lat.field("d%s_phi" % "xyz"[i], dynamic=False) for i in range(nd)]
    for i in range(nd):
        iq = [0, 0, 0]
        iq[i] = 1
        lat.term(g[i], [Mono(1.0, iq=tuple(iq))], [(phi, 1)])
    lat.term(phi, [Mono(-M * a, q2=1), Mono(-M * k, q2=2)], [(phi, 1)], implicit=True)
    lat.term(phi, [Mono(-M * b, q2=1)], [(phi, 3)])
    for i in range(nd):
        lat.term(phi, [Mono(-1.0)], [(v[i], 1), (g[i], 1)])
    for c in range(nd):
        lat.term(v[c], [Mono(-eta, q2=1)], [(v[c], 1)], implicit=True)
        for i in range(nd):
            for j in range(i, nd):
                # -k sum over (i, j) and (j, i) of P_ci (i q_j): delta_ci (i q_j)
                # + (i q_c)(i q_i)(i q_j)/q^2
                merged = {}
                for p_, r_ in ([(i, j)] if i == j else [(i, j), (j, i)]):
                    if p_ == c:
                        iq = [0, 0, 0]
                        iq[r_] += 1
                        key = (0, 0, tuple(iq))
                        merged[key] = merged.get(key, 0.0) - k
                    iq = [0, 0, 0]
                    iq[c] += 1
                    iq[p_] += 1
                    iq[r_] += 1
                    key = (0, 2, tuple(iq))  # equal monomials (the two orders of a mixed pair) add up
                    merged[key] = merged.get(key, 0.0) - k
                monos = [Mono(cf, q2=q2, invq=iv, iq=iq) for (q2, iv, iq), cf in merged.items()]
                lat.term(v[c], monos, [(g[i], 2)] if i == j else [(g[i], 1), (g[j], 1)])
    if D:
        lat.noise(phi, [Mono(D, q2=1)])
    return (phi, *v), tuple(g)
