"""Sakura CPU oracle -- TEST INFRASTRUCTURE ONLY.

ctypes wrapper around ``libsakura_oracle.so`` (plain fp64 C).  Only the tests,
``__graft_entry__.smoke()`` and the benchmark's CPU-baseline leg may import
this package; the HIP library never calls it.  Arrays are numpy float64:
masses [n], positions and velocities [n, 3].
"""
import ctypes
import os

import numpy as np

from .build import LIB, build

SOLVER_KEPLER = 0
SOLVER_KEPLER_LITERAL = 1
SOLVER_DKD = 2

SCHEME_PSI = 0
SCHEME_UNMERGED = 1
SCHEME_TRIPLE_JUMP = 2

ERRORS = {0: "ok", -1: "EINVAL", -2: "ENONFINITE", -3: "ECOLLIDE", -4: "ENOCONV"}


class OracleError(RuntimeError):
    def __init__(self, code, where):
        super().__init__(f"{where}: {ERRORS.get(code, code)}")
        self.code = code


_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = ctypes.CDLL(LIB)
        L.sref_stumpff_c2.restype = ctypes.c_double
        L.sref_stumpff_c2.argtypes = [ctypes.c_double]
        L.sref_stumpff_c3.restype = ctypes.c_double
        L.sref_stumpff_c3.argtypes = [ctypes.c_double]
        L.sref_kepler.argtypes = [ctypes.c_double, ctypes.c_double, _D, _D, _D, _D,
                                  _D, ctypes.POINTER(ctypes.c_int)]
        L.sref_pair_increment.argtypes = [ctypes.c_double, ctypes.c_double,
                                          ctypes.c_double, ctypes.c_double,
                                          _D, _D, _D, _D, ctypes.c_int, _D, _D]
        L.sref_step.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                ctypes.c_double, ctypes.c_int]
        L.sref_step_rows.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int64, _I64, _D, _D]
        L.sref_evolve.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                  ctypes.c_int64, ctypes.c_double, ctypes.c_int]
        L.sref_pair_map.argtypes = [ctypes.c_double] * 6 + [_D] * 6
        L.sref_w_stage.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.sref_evolve_scheme.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                         ctypes.c_int64, ctypes.c_double, ctypes.c_int]
        L.sref_pair_is_close.argtypes = [ctypes.c_double] * 4 + [_D, _D, ctypes.c_double]
        L.sref_step_hybrid.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, _I64]
        L.sref_step_rows_hybrid.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_double, ctypes.c_int64,
                                            _I64, _D, _D]
        L.sref_energy.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double, _D]
        L.sref_row_terms.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int64, _D, _D]
        L.sref_num_threads.restype = ctypes.c_int
        L.sref_set_num_threads.argtypes = [ctypes.c_int]
        L.sref_set_num_threads.restype = None
        L.sref_mlp_forward.argtypes = [_D, ctypes.c_int64, _D, _D]
        L.sref_mlp_loss_grad.argtypes = [_D, ctypes.c_int64, _D, _D, _D, _D]
        L.sref_guess_sample.argtypes = [ctypes.c_double, ctypes.c_double, _D, _D, _D, _D,
                                        _D, ctypes.POINTER(ctypes.c_int)]
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(_D)


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def stumpff_c2(z):
    return lib().sref_stumpff_c2(float(z))


def stumpff_c3(z):
    return lib().sref_stumpff_c3(float(z))


def kepler(tau, mu, x0, w0):
    """Kepler flow (eq. 18).  Returns (x1, w1, coef, iters) with
    coef = (f-1, g-tau, fdot, gdot-1)."""
    x0 = _f64(x0, (3,)).copy()
    w0 = _f64(w0, (3,)).copy()
    x1 = np.empty(3)
    w1 = np.empty(3)
    coef = np.empty(4)
    it = ctypes.c_int(0)
    rc = lib().sref_kepler(float(tau), float(mu), _p(x0), _p(w0), _p(x1), _p(w1),
                           _p(coef), ctypes.byref(it))
    if rc:
        raise OracleError(rc, "sref_kepler")
    return x1, w1, coef, it.value


def pair_increment(tau, G, mi, mj, ri, vi, rj, vj, solver=SOLVER_KEPLER):
    """Relative increments (dr_ij, dv_ij) of the eq. (26) pair map."""
    a = [_f64(x, (3,)).copy() for x in (ri, vi, rj, vj)]
    dr = np.empty(3)
    dv = np.empty(3)
    rc = lib().sref_pair_increment(float(tau), float(G), float(mi), float(mj),
                                   _p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]),
                                   int(solver), _p(dr), _p(dv))
    if rc:
        raise OracleError(rc, "sref_pair_increment")
    return dr, dv


def step(m, r, v, tau, G=1.0, solver=SOLVER_KEPLER):
    """One eq. (27) step; returns new (r, v), inputs untouched."""
    m = _f64(m)
    n = m.shape[0]
    r = _f64(r, (n, 3)).copy()
    v = _f64(v, (n, 3)).copy()
    rc = lib().sref_step(n, _p(m), _p(r), _p(v), float(tau), float(G), int(solver))
    if rc:
        raise OracleError(rc, "sref_step")
    return r, v


def evolve(m, r, v, tau, nsteps, G=1.0, solver=SOLVER_KEPLER):
    m = _f64(m)
    n = m.shape[0]
    r = _f64(r, (n, 3)).copy()
    v = _f64(v, (n, 3)).copy()
    rc = lib().sref_evolve(n, _p(m), _p(r), _p(v), float(tau), int(nsteps),
                           float(G), int(solver))
    if rc:
        raise OracleError(rc, "sref_evolve")
    return r, v


def pair_map(t, cb, ca, G, mi, mj, ri, vi, rj, vj):
    """Relative increments of one pair under back-drift cb, Kepler flow t,
    back-drift ca (eqs. 19a, 19b, 26 are special cases)."""
    a = [_f64(x, (3,)).copy() for x in (ri, vi, rj, vj)]
    dr = np.empty(3)
    dv = np.empty(3)
    rc = lib().sref_pair_map(float(t), float(cb), float(ca), float(G), float(mi), float(mj),
                             _p(a[0]), _p(a[1]), _p(a[2]), _p(a[3]), _p(dr), _p(dv))
    if rc:
        raise OracleError(rc, "sref_pair_map")
    return dr, dv


def w_stage(m, r, v, t, cb, ca, G=1.0):
    """One W stage (eq. 23 with the pair map (t, cb, ca)), no drifts."""
    m = _f64(m)
    n = m.shape[0]
    r = _f64(r, (n, 3)).copy()
    v = _f64(v, (n, 3)).copy()
    rc = lib().sref_w_stage(n, _p(m), _p(r), _p(v), float(t), float(cb), float(ca), float(G))
    if rc:
        raise OracleError(rc, "sref_w_stage")
    return r, v


def evolve_scheme(m, r, v, tau, nsteps, scheme, G=1.0):
    """nsteps steps of a composition scheme (SCHEME_PSI, SCHEME_UNMERGED,
    SCHEME_TRIPLE_JUMP)."""
    m = _f64(m)
    n = m.shape[0]
    r = _f64(r, (n, 3)).copy()
    v = _f64(v, (n, 3)).copy()
    rc = lib().sref_evolve_scheme(n, _p(m), _p(r), _p(v), float(tau), int(nsteps),
                                  float(G), int(scheme))
    if rc:
        raise OracleError(rc, "sref_evolve_scheme")
    return r, v


def pair_is_close(tau, G, mi, mj, X, W, eta):
    """The close-pair test of the hybrid step (Kepler map when True)."""
    X = _f64(X, (3,)).copy()
    W = _f64(W, (3,)).copy()
    return bool(lib().sref_pair_is_close(float(tau), float(G), float(mi), float(mj), _p(X),
                                         _p(W), float(eta)))


def step_hybrid(m, r, v, tau, eta, G=1.0):
    """One hybrid step; returns (r, v, number of Kepler pairs)."""
    m = _f64(m)
    n = m.shape[0]
    r = _f64(r, (n, 3)).copy()
    v = _f64(v, (n, 3)).copy()
    nk = ctypes.c_int64(0)
    rc = lib().sref_step_hybrid(n, _p(m), _p(r), _p(v), float(tau), float(G), float(eta),
                                ctypes.byref(nk))
    if rc:
        raise OracleError(rc, "sref_step_hybrid")
    return r, v, nk.value


def step_rows_hybrid(m, r, v, tau, eta, rows, G=1.0):
    m = _f64(m)
    n = m.shape[0]
    r = _f64(r, (n, 3))
    v = _f64(v, (n, 3))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    ro = np.empty((rows.shape[0], 3))
    vo = np.empty((rows.shape[0], 3))
    rc = lib().sref_step_rows_hybrid(n, _p(m), _p(r), _p(v), float(tau), float(G), float(eta),
                                     rows.shape[0], rows.ctypes.data_as(_I64), _p(ro), _p(vo))
    if rc:
        raise OracleError(rc, "sref_step_rows_hybrid")
    return ro, vo


def step_rows(m, r, v, tau, rows, G=1.0):
    """State after one step for the particles in ``rows`` only."""
    m = _f64(m)
    n = m.shape[0]
    r = _f64(r, (n, 3))
    v = _f64(v, (n, 3))
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    ro = np.empty((rows.shape[0], 3))
    vo = np.empty((rows.shape[0], 3))
    rc = lib().sref_step_rows(n, _p(m), _p(r), _p(v), float(tau), float(G),
                              rows.shape[0], rows.ctypes.data_as(_I64), _p(ro), _p(vo))
    if rc:
        raise OracleError(rc, "sref_step_rows")
    return ro, vo


def row_terms(m, r, v, tau, i, G=1.0):
    """The weighted increments w_ij dr_ij, w_ij dv_ij ([n, 3] each) that row i
    of one step sums."""
    m = _f64(m)
    n = m.shape[0]
    r = _f64(r, (n, 3))
    v = _f64(v, (n, 3))
    dr = np.empty((n, 3))
    dv = np.empty((n, 3))
    rc = lib().sref_row_terms(n, _p(m), _p(r), _p(v), float(tau), float(G), int(i), _p(dr),
                              _p(dv))
    if rc:
        raise OracleError(rc, "sref_row_terms")
    return dr, dv


def energy(m, r, v, G=1.0):
    """Returns dict E, K, U, P, L, Rcm."""
    m = _f64(m)
    n = m.shape[0]
    r = _f64(r, (n, 3))
    v = _f64(v, (n, 3))
    out = np.empty(12)
    rc = lib().sref_energy(n, _p(m), _p(r), _p(v), float(G), _p(out))
    if rc:
        raise OracleError(rc, "sref_energy")
    return {"E": out[0], "K": out[1], "U": out[2], "P": out[3:6].copy(),
            "L": out[6:9].copy(), "Rcm": out[9:12].copy()}


def num_threads():
    return lib().sref_num_threads()


def set_num_threads(n):
    """Threads of the oracle's row loops from now on (results are unchanged)."""
    lib().sref_set_num_threads(int(n))


MLP_PARAMS = 4801


def mlp_forward(params, x):
    """Reference forward pass of the learned-starter network (fp64)."""
    p = _f64(params, (MLP_PARAMS,))
    x = _f64(x).reshape(-1, 8)
    out = np.empty(x.shape[0])
    rc = lib().sref_mlp_forward(_p(p), x.shape[0], _p(x), _p(out))
    if rc:
        raise OracleError(rc, "sref_mlp_forward")
    return out


def mlp_loss_grad(params, x, y):
    """Mean squared error and its gradient (fp64)."""
    p = _f64(params, (MLP_PARAMS,))
    x = _f64(x).reshape(-1, 8)
    y = _f64(y, (x.shape[0],))
    loss = np.empty(1)
    grad = np.empty(MLP_PARAMS)
    rc = lib().sref_mlp_loss_grad(_p(p), x.shape[0], _p(x), _p(y), _p(loss), _p(grad))
    if rc:
        raise OracleError(rc, "sref_mlp_loss_grad")
    return float(loss[0]), grad


def guess_sample(tau, mu, x0, w0, domain):
    """Inputs, domain flag and target of the learned Kepler starter for one
    pair: returns (feat[8], y, in_domain); y is 0 outside the domain."""
    x0 = _f64(x0, (3,)).copy()
    w0 = _f64(w0, (3,)).copy()
    dom = _f64(domain, (4,)).copy()
    feat = np.empty(8)
    y = np.empty(1)
    ind = ctypes.c_int(0)
    rc = lib().sref_guess_sample(float(tau), float(mu), _p(x0), _p(w0), _p(dom), _p(feat),
                                 _p(y), ctypes.byref(ind))
    if rc:
        raise OracleError(rc, "sref_guess_sample")
    return feat, float(y[0]), bool(ind.value)
