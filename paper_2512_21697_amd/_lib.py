"""ctypes binding of libtdde.so (include/tdde.h). Argument marshalling only.

Device buffers are torch tensors on the GPU (complex128 / complex64, contiguous); the library
only sees their data pointers. The library must be built (``python -m paper_2512_21697_amd.build``);
importing this module without it raises, there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtdde.so")

TDDE_OK, TDDE_NOT_CONVERGED, TDDE_BREAKDOWN, TDDE_NONFINITE = 0, 1, 2, 3
GUESS_ZERO, GUESS_PREV, GUESS_GIVEN = 0, 1, 2
PREC_FP64, PREC_MIXED = 0, 1


class Dims(C.Structure):
    _fields_ = [("nr", C.c_int32), ("nang", C.c_int32), ("half_band", C.c_int32), ("batch", C.c_int32),
                ("n_fields", C.c_int32)]


class OperatorDescC(C.Structure):
    _fields_ = [("kappa", C.c_void_p), ("n_h", C.c_int32), ("h_poly", C.c_void_p), ("h_chan", C.c_void_p),
                ("n_s", C.c_int32), ("s_poly", C.c_void_p), ("n_terms", C.c_int32), ("a_rowptr", C.c_void_p),
                ("a_off", C.c_void_p), ("a_col", C.c_void_p), ("a_val", C.c_void_p), ("r_band", C.c_void_p),
                ("kpow", C.c_void_p), ("coef", C.c_void_p), ("field", C.c_void_p)]


class PulseC(C.Structure):
    _fields_ = [("amp", C.c_double), ("T", C.c_double), ("omega", C.c_double), ("phase", C.c_double),
                ("envelope", C.c_int32), ("pad_", C.c_int32)]


class C128(C.Structure):
    _fields_ = [("re", C.c_double), ("im", C.c_double)]


class SolveOpts(C.Structure):
    _fields_ = [("tol", C.c_double), ("max_iter", C.c_int32), ("guess", C.c_int32), ("precond", C.c_int32),
                ("precision", C.c_int32), ("inner_tol", C.c_double), ("max_outer", C.c_int32), ("pad_", C.c_int32)]


class SolveStats(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32), ("matvecs", C.c_int32), ("restarts", C.c_int32),
                ("outer_iters", C.c_int32), ("precs", C.c_int32), ("rel_res", C.c_double),
                ("true_rel_res", C.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


STATS_DTYPE = np.dtype([("status", "<i4"), ("iters", "<i4"), ("matvecs", "<i4"), ("restarts", "<i4"),
                        ("outer_iters", "<i4"), ("precs", "<i4"), ("rel_res", "<f8"), ("true_rel_res", "<f8")])

EXPORTS = ["tdde_create", "tdde_assemble", "tdde_set_dt", "tdde_set_pulses", "tdde_set_field_table", "tdde_eval_pulses", "tdde_set_field", "tdde_apply",
           "tdde_apply_c64", "tdde_precond_apply", "tdde_solve", "tdde_solve_static", "tdde_step", "tdde_spectrum_setup", "tdde_spectrum",
           "tdde_spectrum_error", "tdde_run_batched", "tdde_destroy",
           "tdde_launch_info", "tdde_set_launch", "tdde_set_prec_segment", "tdde_set_split", "tdde_set_prec_storage", "tdde_set_graph", "tdde_status_string", "tdde_last_error", "tdde_debug_phase_marks",
           "tdde_debug_read_marks", "tdde_debug_set_shadow", "tdde_debug_split_timing", "tdde_debug_read_split_timing", "tdde_mlp_create", "tdde_mlp_destroy",
           "tdde_mlp_param_count", "tdde_mlp_set_params", "tdde_mlp_get_params", "tdde_mlp_get_grads",
           "tdde_mlp_forward", "tdde_mlp_backward", "tdde_mlp_adam", "tdde_mlp_set_pulses", "tdde_mlp_guess",
           "tdde_mlp_last_error", "tdde_mlp_fit_skip", "tdde_mlp_set_skip", "tdde_mlp_get_skip"]

_lib = None


def load():
    """Load libtdde.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2512_21697_amd.build`")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "tdde_create": [C.POINTER(Dims), P, C.POINTER(P)],
        "tdde_assemble": [P, C.POINTER(OperatorDescC)],
        "tdde_set_dt": [P, C.c_double],
        "tdde_set_pulses": [P, P],
        "tdde_set_field_table": [P, P, C.c_int32],
        "tdde_eval_pulses": [P, C.c_double, C.c_int32, C.c_int32, P],
        "tdde_set_field": [P, P],
        "tdde_apply": [P, C128, C128, P, P],
        "tdde_apply_c64": [P, C128, C128, P, P],
        "tdde_precond_apply": [P, P, P],
        "tdde_solve": [P, P, P, C.POINTER(SolveOpts), P],
        "tdde_solve_static": [P, P, P, C.POINTER(SolveOpts), P],
        "tdde_spectrum_setup": [P, C.c_int32, P, P, P, P, P, P, C.c_int32],
        "tdde_spectrum": [P, P, P],
        "tdde_spectrum_error": [P, P, P, P],
        "tdde_step": [P, P, C.c_double, P, C.POINTER(SolveOpts), P],
        "tdde_run_batched": [P, P, C.c_double, C.c_int32, C.c_int32, P, P, C.POINTER(SolveOpts), P],
        "tdde_destroy": [P],
        "tdde_launch_info": [P, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
        "tdde_set_launch": [P, C.c_int32],
        "tdde_set_prec_segment": [P, C.c_int32],
        "tdde_set_split": [P, C.c_int32],
        "tdde_set_prec_storage": [P, C.c_int32],
        "tdde_set_graph": [P, C.c_int32],
        "tdde_debug_phase_marks": [P, C.c_int32],
        "tdde_debug_read_marks": [P, P, C.c_int32],
        "tdde_debug_set_shadow": [P, P],
        "tdde_debug_split_timing": [P, C.c_int32],
        "tdde_debug_read_split_timing": [P, P, C.c_int32, P],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.tdde_status_string.argtypes = [C.c_int]
    lib.tdde_status_string.restype = C.c_char_p
    lib.tdde_last_error.argtypes = [P]
    lib.tdde_last_error.restype = C.c_char_p
    msig = {
        "tdde_mlp_create": [C.c_int32, C.c_double, P, C.POINTER(P)],
        "tdde_mlp_destroy": [P],
        "tdde_mlp_set_params": [P, P],
        "tdde_mlp_get_params": [P, P],
        "tdde_mlp_get_grads": [P, P],
        "tdde_mlp_forward": [P, P, C.c_int32, P],
        "tdde_mlp_backward": [P, P, C.c_int32, C.POINTER(C.c_double)],
        "tdde_mlp_adam": [P, C.c_float],
        "tdde_mlp_fit_skip": [P, P, C.c_int32],
        "tdde_mlp_set_skip": [P, P, C.c_double],
        "tdde_mlp_get_skip": [P, P, C.POINTER(C.c_double)],
        "tdde_mlp_set_pulses": [P, P, C.c_int32, C.c_int32],
        "tdde_mlp_guess": [P, C.POINTER(P), C.c_int32, C.c_int64, C.c_int32, C.c_double, C.c_double, P],
    }
    for name, args in msig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = C.c_int
    lib.tdde_mlp_param_count.argtypes = []
    lib.tdde_mlp_param_count.restype = C.c_int64
    lib.tdde_mlp_last_error.argtypes = [P]
    lib.tdde_mlp_last_error.restype = C.c_char_p
    _lib = lib
    return lib


class TddeError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"tdde status {status}: {msg}")
        self.status = status


def _ptr(t):
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("device buffers must be contiguous")
    return C.c_void_p(t.data_ptr())


def _buf(t, n, c64=False):
    """Pointer of a device state buffer after checking dtype, device and element count."""
    import torch
    want = torch.complex64 if c64 else torch.complex128
    if t.dtype != want or not t.is_cuda or t.numel() != n or not t.is_contiguous():
        raise ValueError(f"expected a contiguous CUDA {want} tensor with {n} elements, got "
                         f"{t.dtype} {tuple(t.shape)} on {t.device}")
    return C.c_void_p(t.data_ptr())


def _np(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def solve_opts(tol=1e-12, max_iter=500, guess=GUESS_PREV, precond=0, precision=PREC_FP64, inner_tol=1e-5,
               max_outer=20):
    return SolveOpts(tol, max_iter, guess, precond, precision, inner_tol, max_outer, 0)


class Solver:
    """One library context: operator, workspace, stream."""

    def __init__(self, op, batch: int, stream=None):
        import torch
        self.lib = load()
        self.op = op
        self.batch = batch
        self.nr, self.nang, self.hb = op.nr, op.nang, op.hb
        self.n_fields = op.n_fields
        self.E = op.nang * 2 * op.nr
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        d = Dims(op.nr, op.nang, op.hb, batch, op.n_fields)
        h = C.c_void_p()
        st = self.lib.tdde_create(C.byref(d), C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != TDDE_OK:
            raise TddeError(st, self.lib.tdde_last_error(None).decode())
        self.h = h
        self._assemble(op)

    def _check(self, st, allow=(TDDE_OK,)):
        if st not in allow:
            raise TddeError(st, self.lib.tdde_last_error(self.h).decode())
        return st

    def _assemble(self, op):
        keep = []

        def arr(a, dtype):
            x = _np(a, dtype)
            keep.append(x)
            return x.ctypes.data_as(C.c_void_p)

        nr, nang, nb = op.nr, op.nang, 2 * op.hb + 1

        def need(a, shape, what):
            if tuple(np.shape(a)) != tuple(shape):
                raise ValueError(f"{what}: expected shape {tuple(shape)}, got {tuple(np.shape(a))}")
        need(op.kappa, (nang,), "kappa")
        need(op.h_poly, (op.h_poly.shape[0], 2, 2, nb, nr), "h_poly")
        need(op.s_poly, (op.s_poly.shape[0], 2, 2, nb, nr), "s_poly")
        if op.h_chan is not None:
            need(op.h_chan, (nang, 2, 2, nb, nr), "h_chan")
        for m, t in enumerate(op.terms):
            need(t.a_rowptr, (nang + 1,), f"term {m} a_rowptr")
            need(t.r_band, (2, 2, nb, nr), f"term {m} r_band")
            if len(t.a_col) != len(t.a_val) or int(t.a_rowptr[-1]) != len(t.a_col):
                raise ValueError(f"term {m}: CSR arrays inconsistent")
            if not 0 <= t.field < op.n_fields:
                raise ValueError(f"term {m}: field index out of range")
        desc = OperatorDescC()
        desc.kappa = arr(op.kappa, np.float64)
        desc.n_h = op.h_poly.shape[0]
        desc.h_poly = arr(op.h_poly, np.float64) if desc.n_h else None
        if op.h_chan is not None:
            hc = np.ascontiguousarray(op.h_chan, dtype=np.complex128).view(np.float64)
            desc.h_chan = arr(hc, np.float64)
        desc.n_s = op.s_poly.shape[0]
        desc.s_poly = arr(op.s_poly, np.float64) if desc.n_s else None
        T = len(op.terms)
        desc.n_terms = T
        if T:
            rowptr = np.concatenate([t.a_rowptr.astype(np.int32) for t in op.terms])
            offs = np.zeros(T + 1, dtype=np.int64)
            offs[1:] = np.cumsum([len(t.a_col) for t in op.terms])
            desc.a_rowptr = arr(rowptr, np.int32)
            desc.a_off = arr(offs, np.int64)
            desc.a_col = arr(np.concatenate([t.a_col for t in op.terms]), np.int32)
            desc.a_val = arr(np.concatenate([t.a_val for t in op.terms]), np.float64)
            desc.r_band = arr(np.stack([t.r_band for t in op.terms]), np.float64)
            desc.kpow = arr(np.array([t.kpow for t in op.terms]), np.int32)
            desc.coef = arr(np.array([[t.coef.real, t.coef.imag] for t in op.terms]), np.float64)
            desc.field = arr(np.array([t.field for t in op.terms]), np.int32)
        self._check(self.lib.tdde_assemble(self.h, C.byref(desc)))

    def close(self):
        if getattr(self, "h", None):
            self.lib.tdde_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_dt(self, dt):
        self._check(self.lib.tdde_set_dt(self.h, float(dt)))

    def set_pulses(self, pulses):
        arr = (PulseC * (self.batch * self.n_fields))()
        for b in range(self.batch):
            for m in range(self.n_fields):
                p = pulses[b][m]
                arr[b * self.n_fields + m] = PulseC(p.amp, p.T, p.omega, p.phase, 1 if p.envelope else 0, 0)
        self._check(self.lib.tdde_set_pulses(self.h, C.cast(arr, C.c_void_p)))

    def set_field_table(self, table):
        """Field table [batch][n_rows][n_fields] (row n: the time functions at the midpoint of step n)."""
        t = np.ascontiguousarray(table, dtype=np.float64)
        if t.ndim != 3 or t.shape[0] != self.batch or t.shape[2] != self.n_fields:
            raise ValueError("field table must be [batch][n_rows][n_fields]")
        self._check(self.lib.tdde_set_field_table(self.h, t.ctypes.data_as(C.c_void_p), int(t.shape[1])))

    def eval_pulses(self, t0, step0, n):
        """The pulses evaluated on the device at the midpoints of steps step0 .. step0 + n - 1:
        array [batch][n][n_fields]."""
        out = np.zeros((self.batch, int(n), self.n_fields), dtype=np.float64)
        self._check(self.lib.tdde_eval_pulses(self.h, float(t0), int(step0), int(n), out.ctypes.data_as(C.c_void_p)))
        return out

    def set_field(self, f):
        f = _np(np.asarray(f).reshape(self.batch, self.n_fields), np.float64)
        self._check(self.lib.tdde_set_field(self.h, f.ctypes.data_as(C.c_void_p)))

    def apply(self, x, y, a_s=1.0, a_h=0.0, c64=False):
        fn = self.lib.tdde_apply_c64 if c64 else self.lib.tdde_apply
        n = self.batch * self.E
        self._check(fn(self.h, C128(complex(a_s).real, complex(a_s).imag), C128(complex(a_h).real, complex(a_h).imag),
                       _buf(x, n, c64), _buf(y, n, c64)))

    def precond_apply(self, v, z):
        n = self.batch * self.E
        self._check(self.lib.tdde_precond_apply(self.h, _buf(v, n), _buf(z, n)))

    def solve(self, b, x, opts, stats=True, static=False):
        """tdde_solve, or tdde_solve_static (scratch in the library's static device array) when
        static is true."""
        out = (SolveStats * self.batch)() if stats else None
        n = self.batch * self.E
        fn = self.lib.tdde_solve_static if static else self.lib.tdde_solve
        st = self._check(fn(self.h, _buf(b, n), _buf(x, n), C.byref(opts), C.cast(out, C.c_void_p) if stats else None),
                         allow=(TDDE_OK, TDDE_NOT_CONVERGED, TDDE_BREAKDOWN, TDDE_NONFINITE))
        return st, ([s.as_dict() for s in out] if stats else None)

    def step(self, psi, t, opts, guess=None, stats=True):
        out = (SolveStats * self.batch)() if stats else None
        n = self.batch * self.E
        g = _buf(guess, n) if guess is not None else None
        st = self._check(self.lib.tdde_step(self.h, _buf(psi, n), float(t), g, C.byref(opts),
                                            C.cast(out, C.c_void_p) if stats else None),
                         allow=(TDDE_OK, TDDE_NOT_CONVERGED, TDDE_BREAKDOWN, TDDE_NONFINITE))
        return st, ([s.as_dict() for s in out] if stats else None)

    def run_batched(self, psi, t0, step0, n_chunk, n_steps, opts, stats_dev=None, guess=None):
        ns = _np(n_steps, np.int32)
        if ns.shape != (self.batch,):
            raise ValueError("n_steps must have one entry per instance")
        if stats_dev is not None:
            import torch
            if (stats_dev.dtype != torch.uint8 or not stats_dev.is_cuda or not stats_dev.is_contiguous()
                    or stats_dev.numel() < n_chunk * self.batch * STATS_DTYPE.itemsize):
                raise ValueError("stats_dev must be a contiguous CUDA uint8 tensor of n_chunk*batch*40 bytes")
        g = _buf(guess, self.batch * self.E) if guess is not None else None
        self._check(self.lib.tdde_run_batched(self.h, _buf(psi, self.batch * self.E), float(t0), int(step0),
                                              int(n_chunk), ns.ctypes.data_as(C.c_void_p), g, C.byref(opts),
                                              _ptr(stats_dev)))

    def spectrum_setup(self, blk_of, n_lev, levels, edges, vecs, grid):
        """Eigen-blocks of the photoelectron spectrum (see include/tdde.h: tdde_spectrum_setup)."""
        blk = _np(blk_of, np.int32)
        nl = _np(n_lev, np.int32)
        lv = _np(levels, np.float64)
        ed = _np(edges, np.float64)
        vc = _np(vecs, np.float64)
        gr = _np(grid, np.float64)
        if blk.shape != (self.nang,) or ed.shape != (nl.size, 2) or lv.size != int(nl.sum()) or \
                vc.size != lv.size * 2 * self.nr:
            raise ValueError("spectrum inputs have inconsistent shapes")
        self._spec_ngrid = int(gr.size)
        self._check(self.lib.tdde_spectrum_setup(
            self.h, int(nl.size), blk.ctypes.data_as(C.c_void_p), nl.ctypes.data_as(C.c_void_p),
            lv.ctypes.data_as(C.c_void_p), ed.ctypes.data_as(C.c_void_p), vc.ctypes.data_as(C.c_void_p),
            gr.ctypes.data_as(C.c_void_p), int(gr.size)))

    def spectrum(self, psi, out):
        """dP/dE of every instance into the device float64 tensor out [batch][n_grid]."""
        n = self.batch * self.E
        if str(out.dtype) != "torch.float64" or not out.is_cuda or not out.is_contiguous() or \
                out.numel() != self.batch * self._spec_ngrid:
            raise ValueError("out must be a contiguous device float64 tensor [batch][n_grid]")
        self._check(self.lib.tdde_spectrum(self.h, _buf(psi, n), C.c_void_p(out.data_ptr())))

    def spectrum_error(self, p, q):
        """Trapezoidal integral of |p - q|^2 over the grid, per instance (host array [batch])."""
        for t in (p, q):
            if str(t.dtype) != "torch.float64" or not t.is_cuda or not t.is_contiguous() or \
                    t.numel() != self.batch * self._spec_ngrid:
                raise ValueError("spectra must be contiguous device float64 tensors [batch][n_grid]")
        err = np.zeros(self.batch, dtype=np.float64)
        self._check(self.lib.tdde_spectrum_error(self.h, C.c_void_p(p.data_ptr()), C.c_void_p(q.data_ptr()),
                                                 err.ctypes.data_as(C.c_void_p)))
        return err

    def set_shadow(self, shadow):
        """Test hook: shadow residual of the first BiCGSTAB cycle of later solves (None: r^ = r0).
        The tensor must stay alive while those solves run."""
        self._shadow = shadow
        p = None if shadow is None else _buf(shadow, self.batch * self.E)
        self._check(self.lib.tdde_debug_set_shadow(self.h, p))

    def enable_marks(self, cap):
        self._check(self.lib.tdde_debug_phase_marks(self.h, int(cap)))
        self._marks_cap = int(cap)

    def read_marks(self):
        """Phase timestamps of work-group 0: list of (microseconds since the first mark, phase id)."""
        a = np.zeros(self._marks_cap, dtype=np.uint64)
        self._check(self.lib.tdde_debug_read_marks(self.h, a.ctypes.data_as(C.c_void_p), self._marks_cap))
        a = a[a != 0]
        t = (a >> np.uint64(8)).astype(np.float64) / 100.0  # 100 MHz wall clock -> microseconds
        return list(zip((t - t[0]).tolist(), (a & np.uint64(0xFF)).astype(int).tolist())) if len(a) else []

    def set_launch(self, wg_per_cu: int):
        """At most wg_per_cu persistent work-groups per CU (1..4; 0 = default)."""
        self._check(self.lib.tdde_set_launch(self.h, int(wg_per_cu)))

    def set_graph(self, on: bool):
        """Graph mode: persistent chunks captured once and replayed (needs a non-default stream)."""
        self._check(self.lib.tdde_set_graph(self.h, 1 if on else 0))

    def set_prec_segment(self, min_rows: int):
        """Least rows per preconditioner segment; takes effect at the next set_dt."""
        self._check(self.lib.tdde_set_prec_segment(self.h, int(min_rows)))

    def set_split(self, on: bool):
        """Kernel-per-window solver for FP64 steps with the previous-state guess (True), or one
        persistent launch per call (False, the default)."""
        self._check(self.lib.tdde_set_split(self.h, 1 if on else 0))

    def set_prec_storage(self, bits: int):
        """Preconditioner factors read by the kernel-per-window solver in 64 (default) or 32 bits."""
        self._check(self.lib.tdde_set_prec_storage(self.h, int(bits)))

    def split_timing(self, cap: int):
        """Record the launch durations of the kernel-per-window form's apply kernel v = A p^ for the
        next ``cap`` launches (0 disables)."""
        self._check(self.lib.tdde_debug_split_timing(self.h, int(cap)))

    def read_split_timing(self, cap: int = 65536):
        """Durations (ms) of the recorded launches; starts a new recording."""
        buf = (C.c_float * cap)()
        n = C.c_int32()
        self._check(self.lib.tdde_debug_read_split_timing(self.h, buf, cap, C.byref(n)))
        return list(buf[:n.value])

    def launch_info(self):
        a, b = C.c_int32(), C.c_int32()
        self._check(self.lib.tdde_launch_info(self.h, C.byref(a), C.byref(b)))
        return a.value, b.value


class Net:
    """The learned-guess network of include/tdde_mlp.h (parameters and training scratch on the GPU)."""

    RAW = 16

    def __init__(self, train_rows: int, tau: float, stream=None):
        import torch
        self.lib = load()
        self.train_rows = int(train_rows)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = C.c_void_p()
        st = self.lib.tdde_mlp_create(self.train_rows, float(tau), C.c_void_p(stream.cuda_stream), C.byref(h))
        if st != TDDE_OK:
            raise TddeError(st, "tdde_mlp_create failed")
        self.h = h
        self.n_params = int(self.lib.tdde_mlp_param_count())
        self.batch = None

    def _check(self, st):
        if st != TDDE_OK:
            raise TddeError(st, self.lib.tdde_mlp_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            self.lib.tdde_mlp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        a = _np(flat, np.float32)
        if a.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        self._check(self.lib.tdde_mlp_set_params(self.h, a.ctypes.data_as(C.c_void_p)))

    def get_params(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.lib.tdde_mlp_get_params(self.h, a.ctypes.data_as(C.c_void_p)))
        return a

    def get_grads(self):
        a = np.zeros(self.n_params, dtype=np.float32)
        self._check(self.lib.tdde_mlp_get_grads(self.h, a.ctypes.data_as(C.c_void_p)))
        return a

    def _raw(self, raw):
        import torch
        if raw.dtype != torch.float64 or not raw.is_cuda or raw.dim() != 2 or raw.shape[1] != self.RAW \
                or not raw.is_contiguous() or not 0 < raw.shape[0] <= self.train_rows:
            raise ValueError("raw samples must be a contiguous CUDA float64 [M][16] tensor, M <= train_rows")
        return C.c_void_p(raw.data_ptr()), int(raw.shape[0])

    def forward(self, raw, out):
        import torch
        p, M = self._raw(raw)
        if out.dtype != torch.float32 or not out.is_cuda or out.numel() != 2 * M or not out.is_contiguous():
            raise ValueError("out must be a contiguous CUDA float32 tensor of 2*M values")
        self._check(self.lib.tdde_mlp_forward(self.h, p, M, C.c_void_p(out.data_ptr())))

    def backward(self, raw):
        p, M = self._raw(raw)
        loss = C.c_double()
        self._check(self.lib.tdde_mlp_backward(self.h, p, M, C.byref(loss)))
        return loss.value

    def adam(self, lr):
        self._check(self.lib.tdde_mlp_adam(self.h, float(lr)))

    def fit_skip(self, raw):
        """Least-squares four-step skip on the device (any number of rows)."""
        import torch
        if raw.dtype != torch.float64 or not raw.is_cuda or raw.dim() != 2 or raw.shape[1] != self.RAW \
                or not raw.is_contiguous() or raw.shape[0] <= 0:
            raise ValueError("raw samples must be a contiguous CUDA float64 [M][16] tensor")
        self._check(self.lib.tdde_mlp_fit_skip(self.h, C.c_void_p(raw.data_ptr()), int(raw.shape[0])))

    def set_skip(self, c, sigma):
        """c: complex [2][4]."""
        a = np.zeros((2, 4, 2))
        cc = np.asarray(c)
        a[..., 0], a[..., 1] = cc.real, cc.imag
        a = np.ascontiguousarray(a)
        self._check(self.lib.tdde_mlp_set_skip(self.h, a.ctypes.data_as(C.c_void_p), float(sigma)))

    def get_skip(self):
        a = np.zeros((2, 4, 2))
        sig = C.c_double()
        self._check(self.lib.tdde_mlp_get_skip(self.h, a.ctypes.data_as(C.c_void_p), C.byref(sig)))
        return a[..., 0] + 1j * a[..., 1], sig.value

    def set_pulses(self, pulses):
        batch, nf = len(pulses), len(pulses[0])
        arr = (PulseC * (batch * nf))()
        for b in range(batch):
            for m in range(nf):
                q = pulses[b][m]
                arr[b * nf + m] = PulseC(q.amp, q.T, q.omega, q.phase, 1 if q.envelope else 0, 0)
        self._check(self.lib.tdde_mlp_set_pulses(self.h, C.cast(arr, C.c_void_p), batch, nf))
        self.batch = batch

    def guess(self, hist, E, nr, t_n, dt, out):
        """hist: 4 device complex128 tensors (psi_n .. psi_{n-3}), each [batch * E]."""
        n = self.batch * E
        ptrs = (C.c_void_p * 4)(*[_buf(h, n).value for h in hist])
        self._check(self.lib.tdde_mlp_guess(self.h, ptrs, self.batch, int(E), int(nr), float(t_n), float(dt),
                                            _buf(out, n)))
