"""FP64 CPU oracle for the Lennard-Jones 12-6 short-range force path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check in
``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py`` import
this package.  It shares no code with the HIP library and never calls it.

The arithmetic lives in ``mdlj_oracle.c`` (plain C, binary64, no FMA
contraction); this module only marshals NumPy arrays through ctypes.
What each function computes, with the paper passage it follows, is stated
in the C file.  ``liboracle.so`` is built by ``oracle/build.py`` (the
package's ``build()`` also calls it); it is rebuilt here on first import
when missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = C.POINTER(C.c_double)
_i32 = C.POINTER(C.c_int32)
_i64 = C.POINTER(C.c_int64)
_ci = C.POINTER(C.c_int)


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        from . import build as _b
        _b.build()
    lib = C.CDLL(_LIB_PATH)
    lib.oracle_lj_pair.argtypes = [C.c_double, C.c_double, C.c_double, C.c_double, C.c_int,
                                   _d, _d, _d]
    lib.oracle_lj_pair.restype = None
    lib.oracle_shift.argtypes = [C.c_double, C.c_double, C.c_double, C.c_int]
    lib.oracle_shift.restype = C.c_double
    lib.oracle_mix.argtypes = [C.c_double] * 4 + [_d, _d]
    lib.oracle_mix.restype = None
    lib.oracle_wrap.argtypes = [C.c_double, C.c_double]
    lib.oracle_wrap.restype = C.c_double
    lib.oracle_ncell.argtypes = [C.c_double, C.c_double]
    lib.oracle_ncell.restype = C.c_int
    lib.oracle_bin.argtypes = [C.c_int64, _d, _d, _d, _d, _ci, _i32]
    lib.oracle_bin.restype = None
    force_args = [C.c_int64, _d, _d, _d, _i32, C.c_int, _d, _d, _d, C.c_double, C.c_int,
                  _d, _d, _d, _d, _d, _d]
    lib.oracle_forces_brute.argtypes = force_args
    lib.oracle_forces_brute.restype = C.c_int
    lib.oracle_forces_lc.argtypes = force_args + [C.c_int]
    lib.oracle_forces_lc.restype = C.c_int
    lib.oracle_forces_lc_subset.argtypes = [C.c_int64, _d, _d, _d, _i32, C.c_int, _d, _d, _d,
                                            C.c_double, C.c_int, C.c_int64, _i64, _d, _d, _d,
                                            _d, C.c_int]
    lib.oracle_forces_lc_subset.restype = C.c_int
    lib.oracle_pairs_within.argtypes = [C.c_int64, _d, _d, _d, _d, C.c_double, C.c_int64,
                                        _i64, _i64, _d]
    lib.oracle_pairs_within.restype = C.c_int64
    lib.oracle_vv.argtypes = [C.c_int64, _d, _d, _d, _d, _d, _d, _d, _d, _d, _i32, C.c_int,
                              _d, _d, _d, _d, C.c_double, C.c_int, C.c_double, C.c_int, _d,
                              _d, C.c_int]
    lib.oracle_vv.restype = C.c_int
    lib.oracle_mlp_forward.argtypes = [C.c_int] * 5 + [_d] * 11
    lib.oracle_mlp_forward.restype = None
    lib.oracle_mlp_loss_grad.argtypes = [C.c_int] * 5 + [_d] * 7 + [_i32] + [_d] * 6
    lib.oracle_mlp_loss_grad.restype = C.c_double
    lib.oracle_adam_step.argtypes = [C.c_int64, _d, _d, _d, _d, C.c_int, C.c_double,
                                     C.c_double, C.c_double, C.c_double]
    lib.oracle_adam_step.restype = None
    _lib = lib
    return lib


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a, t=_d):
    return None if a is None else a.ctypes.data_as(t)


class OracleError(RuntimeError):
    pass


def lj_pair(r2, eps=1.0, sig=1.0, rc=2.5, shift=True):
    """(fscal, u, w) for one pair at squared distance r2; F_ij = fscal * d_ij."""
    lib = _load()
    f, u, w = C.c_double(), C.c_double(), C.c_double()
    lib.oracle_lj_pair(float(r2), float(eps), float(sig), float(rc), int(bool(shift)),
                       C.byref(f), C.byref(u), C.byref(w))
    return f.value, u.value, w.value


def mix(eps_a, sig_a, eps_b, sig_b):
    """Lorentz-Berthelot mixed (eps_ab, sig_ab)."""
    lib = _load()
    e, s = C.c_double(), C.c_double()
    lib.oracle_mix(eps_a, sig_a, eps_b, sig_b, C.byref(e), C.byref(s))
    return e.value, s.value


def ncell(L, r):
    return _load().oracle_ncell(float(L), float(r))


def bin_cells(pos, box, nc):
    """Linked-cell index (x fastest) of every particle; pos is (n, 3)."""
    lib = _load()
    pos = _f64(pos)
    x, y, z = (np.ascontiguousarray(pos[:, k]) for k in range(3))
    box = _f64(box)
    nc = np.ascontiguousarray(nc, dtype=np.intc)
    out = np.empty(len(pos), np.int32)
    lib.oracle_bin(len(pos), _p(x), _p(y), _p(z), _p(box), _p(nc, _ci), _p(out, _i32))
    return out


def _species(types, n, eps, sig):
    eps = _f64(np.atleast_1d(eps))
    sig = _f64(np.atleast_1d(sig))
    if types is None:
        types = np.zeros(n, np.int32)
    types = np.ascontiguousarray(types, dtype=np.int32)
    return types, eps, sig


def forces(pos, box, rc, eps=1.0, sig=1.0, types=None, shift=True, method="lc",
           nthreads=0):
    """FP64 forces, per-particle energies and the totals U and W.

    method 'brute' is the O(N^2) sum (section 2.1, Eq. 1); 'lc' is linked
    cells with edge >= rc (section 2.1.1).  Returns dict with keys f (n,3),
    u_i (n,), U, W.
    """
    lib = _load()
    pos = _f64(pos)
    n = len(pos)
    x, y, z = (np.ascontiguousarray(pos[:, k]) for k in range(3))
    types, eps, sig = _species(types, n, eps, sig)
    box = _f64(box)
    fx, fy, fz, ui = (np.zeros(n) for _ in range(4))
    U, W = C.c_double(), C.c_double()
    args = [n, _p(x), _p(y), _p(z), _p(types, _i32), len(eps), _p(eps), _p(sig), _p(box),
            float(rc), int(bool(shift)), _p(fx), _p(fy), _p(fz), _p(ui), C.byref(U),
            C.byref(W)]
    if method == "brute":
        rcode = lib.oracle_forces_brute(*args)
    elif method == "lc":
        rcode = lib.oracle_forces_lc(*args, int(nthreads))
    else:
        raise ValueError(method)
    if rcode:
        raise OracleError(f"oracle forces failed ({rcode})")
    return {"f": np.stack([fx, fy, fz], 1), "u_i": ui, "U": U.value, "W": W.value}


def forces_subset(pos, box, rc, idx, eps=1.0, sig=1.0, types=None, shift=True, nthreads=0):
    """FP64 linked-cell forces and u_i on the particles idx only."""
    lib = _load()
    pos = _f64(pos)
    n = len(pos)
    x, y, z = (np.ascontiguousarray(pos[:, k]) for k in range(3))
    types, eps, sig = _species(types, n, eps, sig)
    box = _f64(box)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    m = len(idx)
    fx, fy, fz, ui = (np.zeros(m) for _ in range(4))
    rcode = lib.oracle_forces_lc_subset(n, _p(x), _p(y), _p(z), _p(types, _i32), len(eps),
                                        _p(eps), _p(sig), _p(box), float(rc),
                                        int(bool(shift)), m, _p(idx, _i64), _p(fx), _p(fy),
                                        _p(fz), _p(ui), int(nthreads))
    if rcode:
        raise OracleError(f"oracle subset forces failed ({rcode})")
    return {"f": np.stack([fx, fy, fz], 1), "u_i": ui}


def pairs_within(pos, box, rmax, cap=None):
    """All unordered pairs (i<j) with r^2 < rmax^2: (pi, pj, r2)."""
    lib = _load()
    pos = _f64(pos)
    n = len(pos)
    x, y, z = (np.ascontiguousarray(pos[:, k]) for k in range(3))
    box = _f64(box)
    if cap is None:
        cnt = lib.oracle_pairs_within(n, _p(x), _p(y), _p(z), _p(box), float(rmax), 0,
                                      None, None, None)
        if cnt < 0:
            raise OracleError(f"oracle pairs failed ({cnt})")
        cap = cnt
    pi = np.empty(cap, np.int64)
    pj = np.empty(cap, np.int64)
    r2 = np.empty(cap)
    cnt = lib.oracle_pairs_within(n, _p(x), _p(y), _p(z), _p(box), float(rmax), cap,
                                  _p(pi, _i64), _p(pj, _i64), _p(r2))
    if cnt < 0 or cnt > cap:
        raise OracleError(f"oracle pairs failed ({cnt})")
    return pi[:cnt], pj[:cnt], r2[:cnt]


def vv(pos, vel, box, rc, dt, nsteps, eps=1.0, sig=1.0, mass=1.0, types=None, shift=True,
       nthreads=0):
    """Velocity-Verlet trajectory; returns (pos, vel, f, epot[nsteps+1], ekin[nsteps+1])."""
    lib = _load()
    pos = _f64(pos).copy()
    vel = _f64(vel).copy()
    n = len(pos)
    x, y, z = (np.ascontiguousarray(pos[:, k]) for k in range(3))
    vx, vy, vz = (np.ascontiguousarray(vel[:, k]) for k in range(3))
    types, eps, sig = _species(types, n, eps, sig)
    mass = _f64(np.broadcast_to(np.atleast_1d(mass), eps.shape))
    box = _f64(box)
    fx, fy, fz = (np.zeros(n) for _ in range(3))
    ep = np.zeros(nsteps + 1)
    ek = np.zeros(nsteps + 1)
    rcode = lib.oracle_vv(n, _p(x), _p(y), _p(z), _p(vx), _p(vy), _p(vz), _p(fx), _p(fy),
                          _p(fz), _p(types, _i32), len(eps), _p(eps), _p(sig), _p(mass),
                          _p(box), float(rc), int(bool(shift)), float(dt), int(nsteps),
                          _p(ep), _p(ek), int(nthreads))
    if rcode:
        raise OracleError(f"oracle vv failed ({rcode})")
    return (np.stack([x, y, z], 1), np.stack([vx, vy, vz], 1), np.stack([fx, fy, fz], 1),
            ep, ek)


def mlp_forward(params, X):
    """params = (W1, b1, W2, b2, W3, b3), W as [out][in]; returns (h1, h2, logits, probs)."""
    lib = _load()
    W1, b1, W2, b2, W3, b3 = (_f64(p) for p in params)
    X = _f64(np.atleast_2d(X))
    B, din = X.shape
    dh1, dh2, k = W1.shape[0], W2.shape[0], W3.shape[0]
    H1 = np.zeros((B, dh1))
    H2 = np.zeros((B, dh2))
    Z = np.zeros((B, k))
    P = np.zeros((B, k))
    lib.oracle_mlp_forward(B, din, dh1, dh2, k, _p(W1), _p(b1), _p(W2), _p(b2), _p(W3),
                           _p(b3), _p(X), _p(H1), _p(H2), _p(Z), _p(P))
    return H1, H2, Z, P


def mlp_loss_grad(params, X, labels):
    """Mean cross-entropy and its gradients (same shapes as params)."""
    lib = _load()
    W1, b1, W2, b2, W3, b3 = (_f64(p) for p in params)
    X = _f64(np.atleast_2d(X))
    B, din = X.shape
    dh1, dh2, k = W1.shape[0], W2.shape[0], W3.shape[0]
    labels = np.ascontiguousarray(labels, dtype=np.int32)
    grads = [np.zeros_like(p) for p in (W1, b1, W2, b2, W3, b3)]
    loss = lib.oracle_mlp_loss_grad(B, din, dh1, dh2, k, _p(W1), _p(b1), _p(W2), _p(b2),
                                    _p(W3), _p(b3), _p(X), _p(labels, _i32),
                                    *[_p(g) for g in grads])
    return loss, grads


def adam_step(w, g, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step in place on float64 arrays w, m, v (g read only)."""
    lib = _load()
    for a in (w, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(g)
    lib.oracle_adam_step(w.size, _p(w), _p(g), _p(m), _p(v), int(t), lr, b1, b2, eps)
