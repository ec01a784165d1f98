"""Python binding of libsakura.so (include/sakura.h): argument marshalling only.

Every step of the integrator runs in the HIP kernels of the library.  torch is
used for device memory and streams: m, r, v are float64 CUDA tensors of shape
[n], [n, 3], [n, 3]; r and v are updated in place on the current stream.
There is no CPU path: if the library is not built, importing raises.
"""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsakura.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sakura.h")

OK, EINVAL, ENONFINITE, ECOLLIDE, ENOCONV, EHIP, ENOMEM, ENOMODEL = 0, -1, -2, -3, -4, -5, -6, -7
ERROR_NAMES = {0: "OK", -1: "EINVAL", -2: "ENONFINITE", -3: "ECOLLIDE", -4: "ENOCONV",
               -5: "EHIP", -6: "ENOMEM", -7: "ENOMODEL"}
GUESS_ANALYTIC, GUESS_LEARNED = 0, 1
SCHEME_PSI, SCHEME_UNMERGED, SCHEME_TRIPLE_JUMP = 0, 1, 2
NOALLOC_MAX_N = 4096


class SakuraError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


class Opts(ctypes.Structure):
    _fields_ = [("guess", ctypes.c_int), ("kepler_rtol", ctypes.c_double),
                ("max_iter", ctypes.c_int), ("histogram", ctypes.c_int),
                ("tile_override", ctypes.c_int), ("row_strip", ctypes.c_int)]


class Stats(ctypes.Structure):
    _fields_ = [("pair_solves", ctypes.c_uint64), ("iters_total", ctypes.c_uint64),
                ("fallbacks", ctypes.c_uint64), ("iters_max", ctypes.c_uint32),
                ("hist", ctypes.c_uint32 * 32), ("pair_kernel_ms", ctypes.c_double),
                ("call_ms", ctypes.c_double), ("pair_launches", ctypes.c_int64),
                ("failed_step", ctypes.c_int64), ("guess_domain_pairs", ctypes.c_uint64),
                ("guess_domain_iters", ctypes.c_uint64), ("guess_learned", ctypes.c_uint64),
                ("guess_restarts", ctypes.c_uint64), ("pair_kicks", ctypes.c_uint64),
                ("max_rel_residual", ctypes.c_double)]

    def to_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "hist"}
        d["hist"] = list(self.hist)
        return d


MLP_PARAMS = 4801
HARVEST_ROW = 12


class GuessModel(ctypes.Structure):
    """sakura_guess_model: fp32 parameters W1[64][8], b1, W2[64][64], b2, W3, b3,
    input/output scaling and the domain {tau_lo, tau_hi, b_lo, e_hi}."""
    _fields_ = [("params", ctypes.c_float * MLP_PARAMS), ("in_shift", ctypes.c_float * 8),
                ("in_scale", ctypes.c_float * 8), ("out_shift", ctypes.c_float),
                ("out_scale", ctypes.c_float), ("domain", ctypes.c_double * 4)]

    def to_dict(self):
        import numpy as np
        return {"params": np.ctypeslib.as_array(self.params).copy(),
                "in_shift": list(self.in_shift), "in_scale": list(self.in_scale),
                "out_shift": self.out_shift, "out_scale": self.out_scale,
                "domain": list(self.domain)}

    @classmethod
    def from_dict(cls, d):
        m = cls()
        for k, v in enumerate(d["params"]):
            m.params[k] = float(v)
        for k in range(8):
            m.in_shift[k] = float(d["in_shift"][k])
            m.in_scale[k] = float(d["in_scale"][k])
        m.out_shift = float(d["out_shift"])
        m.out_scale = float(d["out_scale"])
        for k in range(4):
            m.domain[k] = float(d["domain"][k])
        return m


class FitOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_float),
                ("lr_final", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("val_fraction", ctypes.c_double)]


def declared_functions():
    """Names of the functions include/sakura.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sakura_[a-z_]+)\s*\(", text)))


def load_library():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(the Sakura step has no CPU implementation)")
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    L.sakura_create.argtypes = [ctypes.POINTER(P), ctypes.c_int, ctypes.POINTER(Opts)]
    L.sakura_create.restype = ctypes.c_int
    L.sakura_destroy.argtypes = [P]
    L.sakura_destroy.restype = None
    L.sakura_step.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_double,
                              P, ctypes.POINTER(Stats)]
    L.sakura_step.restype = ctypes.c_int
    L.sakura_evolve.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_double, ctypes.c_int64,
                                ctypes.c_double, P, ctypes.POINTER(Stats)]
    L.sakura_evolve.restype = ctypes.c_int
    L.sakura_evolve_noalloc.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_double,
                                        ctypes.c_int64, ctypes.c_double, P,
                                        ctypes.POINTER(Stats)]
    L.sakura_evolve_noalloc.restype = ctypes.c_int
    L.sakura_evolve_scheme.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_double,
                                       ctypes.c_int64, ctypes.c_double, ctypes.c_int, P,
                                       ctypes.POINTER(Stats)]
    L.sakura_evolve_scheme.restype = ctypes.c_int
    L.sakura_set_hybrid.argtypes = [P, ctypes.c_double]
    L.sakura_set_hybrid.restype = ctypes.c_int
    L.sakura_energy.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_double), P]
    L.sakura_energy.restype = ctypes.c_int
    L.sakura_batch_evolve.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), P, P, P,
                                      P, ctypes.c_int64, ctypes.c_double, P,
                                      ctypes.POINTER(Stats)]
    L.sakura_batch_evolve.restype = ctypes.c_int
    L.sakura_batch_set_policy.argtypes = [P, ctypes.c_int, ctypes.c_int, ctypes.c_int]
    L.sakura_batch_set_policy.restype = ctypes.c_int
    L.sakura_batch_set_group.argtypes = [P, ctypes.c_int, ctypes.c_int]
    L.sakura_batch_set_group.restype = ctypes.c_int
    L.sakura_batch_set_width.argtypes = [P, ctypes.c_int, ctypes.c_int]
    L.sakura_batch_set_width.restype = ctypes.c_int
    L.sakura_autotune_batch.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64), P, P, P,
                                        P, ctypes.c_int64, ctypes.c_double, P,
                                        ctypes.POINTER(ctypes.c_double)]
    L.sakura_autotune_batch.restype = ctypes.c_int
    L.sakura_batch_table_save.argtypes = [P, ctypes.c_char_p]
    L.sakura_batch_table_save.restype = ctypes.c_int
    L.sakura_batch_table_load.argtypes = [P, ctypes.c_char_p]
    L.sakura_batch_table_load.restype = ctypes.c_int
    L.sakura_last_error.argtypes = [P]
    L.sakura_last_error.restype = ctypes.c_char_p
    D4 = ctypes.POINTER(ctypes.c_double)
    L.sakura_set_guess_model.argtypes = [P, P, ctypes.c_size_t]
    L.sakura_set_guess.argtypes = [P, ctypes.c_int]
    L.sakura_harvest_begin.argtypes = [P, P, ctypes.c_int64, D4]
    L.sakura_harvest_end.argtypes = [P, ctypes.POINTER(ctypes.c_int64)]
    L.sakura_guess_eval.argtypes = [P, ctypes.c_int64, P, P, P, P, P, P, P, P]
    L.sakura_mlp_forward.argtypes = [P, P, ctypes.c_int64, P, P, P]
    L.sakura_mlp_loss_grad.argtypes = [P, P, ctypes.c_int64, P, P, P, D4, P]
    L.sakura_mlp_fit.argtypes = [P, P, ctypes.c_int64, D4, ctypes.POINTER(FitOpts),
                                 ctypes.POINTER(GuessModel), ctypes.POINTER(ctypes.c_float), P]
    for f in ("sakura_set_guess_model", "sakura_set_guess", "sakura_harvest_begin",
              "sakura_harvest_end", "sakura_guess_eval", "sakura_mlp_forward",
              "sakura_mlp_loss_grad", "sakura_mlp_fit"):
        getattr(L, f).restype = ctypes.c_int
    return L


_LIB = None


def lib():
    global _LIB
    if _LIB is None:
        _LIB = load_library()
    return _LIB


def _check_state(m, r, v):
    import torch
    for name, t in (("m", m), ("r", r), ("v", v)):
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError(f"{name} must be a float64 CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    n = m.shape[0]
    if m.dim() != 1 or tuple(r.shape) != (n, 3) or tuple(v.shape) != (n, 3):
        raise ValueError("shapes must be m [n], r [n, 3], v [n, 3]")
    if not (m.device == r.device == v.device):
        raise ValueError("m, r, v must be on one device")
    return n


class Sakura:
    """A library handle bound to one GPU."""

    def __init__(self, device: int = 0, guess: int = GUESS_ANALYTIC, kepler_rtol: float = 0.0,
                 max_iter: int = 0, histogram: bool = False, tile_override: int = 0,
                 row_strip: int = 0):
        self._lib = lib()
        self.device = device
        h = ctypes.c_void_p()
        o = Opts(guess, kepler_rtol, max_iter, int(bool(histogram)), int(tile_override),
                 int(row_strip))
        rc = self._lib.sakura_create(ctypes.byref(h), device, ctypes.byref(o))
        if rc != OK:
            raise SakuraError(rc, "sakura_create failed")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._lib.sakura_destroy(self._h)
            self._h = None

    __del__ = close

    def _raise(self, rc):
        msg = self._lib.sakura_last_error(self._h)
        raise SakuraError(rc, msg.decode() if msg else "")

    def _state(self, m, r, v):
        n = _check_state(m, r, v)
        if m.device.index != self.device:
            raise ValueError(f"m, r, v are on {m.device}; the handle is bound to "
                             f"cuda:{self.device}")
        return n

    @staticmethod
    def _stream(t):
        import torch
        return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)

    def evolve(self, m, r, v, dt: float, nsteps: int, G: float = 1.0, stats: bool = False):
        """nsteps steps of eqs. (27a-d); r, v updated in place.  Returns the
        stats dict when stats=True."""
        n = self._state(m, r, v)
        st = Stats()
        rc = self._lib.sakura_evolve(self._h, n, ctypes.c_void_p(m.data_ptr()),
                                     ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                     float(dt), int(nsteps), float(G), self._stream(m),
                                     ctypes.byref(st) if stats else None)
        if rc != OK:
            self._raise(rc)
        return st.to_dict() if stats else None

    def evolve_noalloc(self, m, r, v, dt: float, nsteps: int, G: float = 1.0,
                       stats: bool = False):
        """sakura_evolve on the library's static scratch (no device allocation;
        n <= NOALLOC_MAX_N; calls on one device must not overlap)."""
        n = self._state(m, r, v)
        st = Stats()
        rc = self._lib.sakura_evolve_noalloc(self._h, n, ctypes.c_void_p(m.data_ptr()),
                                             ctypes.c_void_p(r.data_ptr()),
                                             ctypes.c_void_p(v.data_ptr()), float(dt),
                                             int(nsteps), float(G), self._stream(m),
                                             ctypes.byref(st) if stats else None)
        if rc != OK:
            self._raise(rc)
        return st.to_dict() if stats else None

    def evolve_scheme(self, m, r, v, dt: float, nsteps: int, scheme: int, G: float = 1.0,
                      stats: bool = False):
        """nsteps steps of a composition of the step (SCHEME_PSI, SCHEME_UNMERGED,
        SCHEME_TRIPLE_JUMP); r, v updated in place."""
        n = self._state(m, r, v)
        st = Stats()
        rc = self._lib.sakura_evolve_scheme(self._h, n, ctypes.c_void_p(m.data_ptr()),
                                            ctypes.c_void_p(r.data_ptr()),
                                            ctypes.c_void_p(v.data_ptr()), float(dt),
                                            int(nsteps), float(G), int(scheme), self._stream(m),
                                            ctypes.byref(st) if stats else None)
        if rc != OK:
            self._raise(rc)
        return st.to_dict() if stats else None

    def set_hybrid(self, eta: float):
        """Close-pair hybrid threshold (0: every pair by the Kepler map)."""
        self._ok(self._lib.sakura_set_hybrid(self._h, float(eta)))

    def step(self, m, r, v, dt: float, G: float = 1.0, stats: bool = False):
        n = self._state(m, r, v)
        st = Stats()
        rc = self._lib.sakura_step(self._h, n, ctypes.c_void_p(m.data_ptr()),
                                   ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                   float(dt), float(G), self._stream(m),
                                   ctypes.byref(st) if stats else None)
        if rc != OK:
            self._raise(rc)
        return st.to_dict() if stats else None

    def _batch_args(self, offsets, m, r, v, dt):
        import numpy as np
        import torch
        off = np.ascontiguousarray(offsets, dtype=np.int64)
        nsys = off.shape[0] - 1
        n = self._state(m, r, v)
        if nsys < 1 or off[0] != 0 or off[-1] != n:
            raise ValueError("offsets must start at 0 and end at len(m)")
        if not (isinstance(dt, torch.Tensor) and dt.dtype == torch.float64 and dt.is_cuda
                and dt.device == m.device and dt.is_contiguous() and tuple(dt.shape) == (nsys,)):
            raise TypeError("dt must be a contiguous float64 CUDA tensor of shape [nsys] "
                            "on the device of m")
        return off, nsys

    def batch_evolve(self, offsets, m, r, v, dt, nsteps: int, G: float = 1.0, stats: bool = False):
        """nsteps steps of every system of a CSR ensemble (offsets: host int64
        [nsys+1]; dt: per-system steps, CUDA float64 [nsys])."""
        off, nsys = self._batch_args(offsets, m, r, v, dt)
        st = Stats()
        rc = self._lib.sakura_batch_evolve(
            self._h, nsys, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(r.data_ptr()),
            ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(dt.data_ptr()), int(nsteps),
            float(G), self._stream(m), ctypes.byref(st) if stats else None)
        if rc != OK:
            self._raise(rc)
        return st.to_dict() if stats else None

    def batch_set_policy(self, policy: int = 0, waves_per_cu: int = 8, use_graph: bool = True):
        rc = self._lib.sakura_batch_set_policy(self._h, policy, waves_per_cu, int(bool(use_graph)))
        if rc != OK:
            self._raise(rc)

    def batch_set_group(self, n: int, lanes: int):
        """Lanes used by systems of exactly n particles."""
        self._ok(self._lib.sakura_batch_set_group(self._h, int(n), int(lanes)))

    def batch_set_width(self, n: int, waves: int):
        """Wavefronts per work item (1, 2 or 4) for systems of exactly n particles."""
        self._ok(self._lib.sakura_batch_set_width(self._h, int(n), int(waves)))

    def autotune_batch(self, offsets, m, r, v, dt, probe_steps: int = 8, G: float = 1.0):
        """Pick the fastest packing policy and grid size for this ensemble
        (r, v are not modified).  Returns the best probe time in ms."""
        off, nsys = self._batch_args(offsets, m, r, v, dt)
        best = ctypes.c_double(0.0)
        rc = self._lib.sakura_autotune_batch(
            self._h, nsys, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
            ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(r.data_ptr()),
            ctypes.c_void_p(v.data_ptr()), ctypes.c_void_p(dt.data_ptr()), int(probe_steps),
            float(G), self._stream(m), ctypes.byref(best))
        if rc != OK:
            self._raise(rc)
        return best.value

    def batch_table_save(self, path):
        """Write the handle's packing table (autotuned entries) to a text file."""
        self._ok(self._lib.sakura_batch_table_save(self._h, str(path).encode()))

    def batch_table_load(self, path):
        """Merge a packing table file into the handle's and apply this device's
        entries."""
        self._ok(self._lib.sakura_batch_table_load(self._h, str(path).encode()))

    def energy(self, m, r, v, G: float = 1.0):
        """{E, K, U, P, L, Rcm} of eqs. (1-3), computed on the GPU."""
        n = self._state(m, r, v)
        out = (ctypes.c_double * 12)()
        rc = self._lib.sakura_energy(self._h, n, ctypes.c_void_p(m.data_ptr()),
                                     ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(v.data_ptr()),
                                     float(G), out, self._stream(m))
        if rc != OK:
            self._raise(rc)
        o = list(out)
        return {"E": o[0], "K": o[1], "U": o[2], "P": o[3:6], "L": o[6:9], "Rcm": o[9:12]}

    # ---- learned Kepler starter -------------------------------------------

    def _ok(self, rc):
        if rc != OK:
            self._raise(rc)

    def set_guess_model(self, model):
        """Load a GuessModel (or a dict from GuessModel.to_dict); None unloads."""
        if model is None:
            self._ok(self._lib.sakura_set_guess_model(self._h, None, 0))
            return
        if isinstance(model, dict):
            model = GuessModel.from_dict(model)
        self._ok(self._lib.sakura_set_guess_model(self._h, ctypes.cast(ctypes.byref(model),
                                                                       ctypes.c_void_p),
                                                  ctypes.sizeof(model)))

    def set_guess(self, guess: int):
        self._ok(self._lib.sakura_set_guess(self._h, int(guess)))

    def harvest_begin(self, rows, domain):
        """Start recording harvest rows into `rows` (CUDA float32 [cap, 12])."""
        import torch
        if not (isinstance(rows, torch.Tensor) and rows.dtype == torch.float32 and rows.is_cuda
                and rows.is_contiguous() and rows.dim() == 2 and rows.shape[1] == HARVEST_ROW):
            raise TypeError("rows must be a contiguous CUDA float32 tensor [cap, 12]")
        dom = (ctypes.c_double * 4)(*[float(x) for x in domain])
        self._ok(self._lib.sakura_harvest_begin(self._h, ctypes.c_void_p(rows.data_ptr()),
                                                rows.shape[0], dom))

    def harvest_end(self):
        """Stop recording; returns the number of rows produced (including any
        dropped beyond the buffer's capacity)."""
        c = ctypes.c_int64(0)
        self._ok(self._lib.sakura_harvest_end(self._h, ctypes.byref(c)))
        return c.value

    def guess_eval(self, tau, mu, x0, w0):
        """The pair kernels' root search on independent problems (CUDA float64
        tau [n], mu [n], x0 [n, 3], w0 [n, 3]).  Returns (s_start, s_root, info)."""
        import torch
        n = tau.shape[0]
        for t in (tau, mu, x0, w0):
            if not (t.dtype == torch.float64 and t.is_cuda and t.is_contiguous()):
                raise TypeError("inputs must be contiguous CUDA float64 tensors")
        if tuple(mu.shape) != (n,) or tuple(x0.shape) != (n, 3) or tuple(w0.shape) != (n, 3):
            raise ValueError("shapes must be tau [n], mu [n], x0 [n, 3], w0 [n, 3]")
        s0 = torch.empty(n, dtype=torch.float64, device=tau.device)
        s1 = torch.empty_like(s0)
        info = torch.empty(n, dtype=torch.int32, device=tau.device)
        ptr = lambda t: ctypes.c_void_p(t.data_ptr())
        self._ok(self._lib.sakura_guess_eval(self._h, n, ptr(tau), ptr(mu), ptr(x0), ptr(w0),
                                             ptr(s0), ptr(s1), ptr(info), self._stream(tau)))
        return s0, s1, info

    def mlp_forward(self, params, x):
        """Network output (fp32 training kernels) for scaled inputs x [b, 8]."""
        import torch
        out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        self._ok(self._lib.sakura_mlp_forward(self._h, ctypes.c_void_p(params.data_ptr()),
                                              x.shape[0], ctypes.c_void_p(x.data_ptr()),
                                              ctypes.c_void_p(out.data_ptr()), self._stream(x)))
        return out

    def mlp_loss_grad(self, params, x, y):
        """Mean squared error and its gradient (fp32 training kernels)."""
        import torch
        grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
        loss = ctypes.c_double(0.0)
        self._ok(self._lib.sakura_mlp_loss_grad(
            self._h, ctypes.c_void_p(params.data_ptr()), x.shape[0],
            ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
            ctypes.c_void_p(grad.data_ptr()), ctypes.byref(loss), self._stream(x)))
        return loss.value, grad

    def mlp_fit(self, rows, domain, epochs=20, batch=4096, lr=3e-3, lr_final=3e-5, seed=1,
                val_fraction=0.05):
        """Train the starter network on harvested rows (CUDA float32 [n, 12]).
        Returns (GuessModel, list of held-out losses per epoch)."""
        model = GuessModel()
        o = FitOpts(int(epochs), int(batch), float(lr), float(lr_final), int(seed),
                    float(val_fraction))
        dom = (ctypes.c_double * 4)(*[float(x) for x in domain])
        hist = (ctypes.c_float * max(1, int(epochs)))()
        self._ok(self._lib.sakura_mlp_fit(self._h, ctypes.c_void_p(rows.data_ptr()),
                                          rows.shape[0], dom, ctypes.byref(o),
                                          ctypes.byref(model), hist, self._stream(rows)))
        return model, list(hist)
