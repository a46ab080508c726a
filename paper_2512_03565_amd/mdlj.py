"""Thin ctypes binding of libmdlj (the C ABI in include/mdlj.h).

Argument marshalling only: every step of the force path runs in the HIP
library.  Functions carry the C names; ``System`` is a small convenience
wrapper used by the tests and the benchmark.  Device arrays are torch CUDA
(HIP) tensors passed by ``data_ptr()``; host arrays are NumPy arrays.
There is no CPU fallback: importing this module fails if ``libmdlj.so`` has
not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmdlj.so")

MDLJ_OK = 0
STATUS = {0: "OK", -1: "ERR_ARG", -2: "ERR_STATE", -3: "ERR_HIP", -4: "ERR_NOMEM",
          -5: "ERR_OVERFLOW", -6: "ERR_NONFINITE", -7: "ERR_GEOMETRY", -8: "ERR_NOTFOUND"}
MEM_HOST, MEM_DEVICE = 0, 1
NBR_LC, NBR_VL, NBR_VCL = 0, 1, 2
ORD_I_PER_LANE, ORD_CLUSTER_TILE, ORD_WAVE_PER_I = 0, 1, 2
PREC_F32PAIR_F64ACC, PREC_F64 = 0, 1
TUNE_FIXED, TUNE_EXHAUSTIVE, TUNE_LEARNED, TUNE_EARLY_STOP = 0, 1, 2, 3
METRIC_TIME, METRIC_ENERGY = 0, 1
NBR_NAMES = {0: "LC", 1: "VL", 2: "VCL"}
ORD_NAMES = {0: "i-per-lane", 1: "cluster-tile", 2: "wave-per-i"}


class mdlj_config(C.Structure):
    _fields_ = [("nbr_algo", C.c_int32), ("order", C.c_int32), ("tile_i", C.c_int32),
                ("tile_j", C.c_int32), ("cluster_size", C.c_int32), ("newton3", C.c_int32),
                ("staged", C.c_int32), ("swap", C.c_int32)]

    def astuple(self):
        return (self.nbr_algo, self.order, self.tile_i, self.tile_j, self.cluster_size,
                self.newton3, self.staged, self.swap)

    def __repr__(self):
        return config_name(self)


def config_name(c) -> str:
    t = c.astuple() if hasattr(c, "astuple") else tuple(c)
    t = tuple(t) + (0,) * (8 - len(t))
    nb, o, ti, tj, m, n3, st, sw = t
    s = NBR_NAMES[nb] + (str(m) if nb == NBR_VCL else "") + "/" + ORD_NAMES[o]
    if o == ORD_I_PER_LANE and nb == NBR_LC and not n3:
        s += f"/k{ti}"
    elif o != ORD_I_PER_LANE:
        s += f"/{ti}x{tj}"
        if nb == NBR_VCL and 0 < ti * tj < 64:
            # cluster pairs per wavefront
            s += f"x{64 // (ti * tj)}"
    return s + ("/n3" if n3 else "") + ("/lds" if st else "") + ("/swap" if sw else "")


class MdljError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with paper_2512_03565_amd/build.py "
                      "(there is no CPU fallback)")

# torch ships its own HIP runtime under the same soname (libamdhip64.so.7).
# Loading torch first makes libmdlj bind to that runtime, so the process
# holds one HIP runtime and torch streams and tensors are valid handles for
# the library.  Loading libmdlj first would pull in a second runtime.
import torch  # noqa: E402,F401

lib = C.CDLL(LIB_PATH)
_vp = C.c_void_p
_d = C.POINTER(C.c_double)
_ctxp = C.c_void_p

_SIGS = {
    "mdlj_create": [C.POINTER(_ctxp), C.c_int64, _vp, _vp, _vp, _vp, C.c_int32, C.c_int32, _vp],
    "mdlj_destroy": [_ctxp],
    "mdlj_set_box": [_ctxp, C.c_double, C.c_double, C.c_double],
    "mdlj_set_cutoff": [_ctxp, C.c_double],
    "mdlj_set_skin": [_ctxp, C.c_double, C.c_int32],
    "mdlj_set_species": [_ctxp, C.c_int32, C.c_double, C.c_double],
    "mdlj_set_energy_shift": [_ctxp, C.c_int32],
    "mdlj_set_pruning": [_ctxp, C.c_int32],
    "mdlj_pruning_state": [_ctxp, C.POINTER(C.c_int32), C.POINTER(C.c_int64)],
    "mdlj_set_precision": [_ctxp, C.c_int32],
    "mdlj_set_positions": [_ctxp, _vp, _vp, _vp, C.c_int32],
    "mdlj_get_positions": [_ctxp, _vp, _vp, _vp, C.c_int32],
    "mdlj_set_config": [_ctxp, C.POINTER(mdlj_config)],
    "mdlj_get_config": [_ctxp, C.POINTER(mdlj_config)],
    "mdlj_config_count": [_ctxp, C.POINTER(C.c_int32)],
    "mdlj_config_at": [_ctxp, C.c_int32, C.POINTER(mdlj_config)],
    "mdlj_rebuild_neighbors": [_ctxp],
    "mdlj_compute_forces": [_ctxp, _vp, _vp, _vp, C.c_int32, _d, _d],
    "mdlj_count_pairs": [_ctxp, C.POINTER(C.c_int64)],
    "mdlj_neighbor_stats": [_ctxp, C.POINTER(C.c_int64), C.POINTER(C.c_int32),
                            C.POINTER(C.c_int64)],
    "mdlj_tune": [_ctxp, C.c_int32, C.c_int32, C.POINTER(mdlj_config), _d],
    "mdlj_tune_results": [_ctxp, _d, C.c_int32, C.POINTER(C.c_int32)],
    "mdlj_tune_taken": [_ctxp, C.POINTER(C.c_int32), C.c_int32, C.POINTER(C.c_int32)],
    "mdlj_tune_select_early": [_d, C.c_int32, C.c_int32, C.POINTER(C.c_int32), C.c_double,
                               C.c_double, _d, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
    "mdlj_step_vv": [_ctxp, _vp, _vp, _vp, C.c_double, C.c_int32],
    "mdlj_set_mass": [_ctxp, C.c_int32, C.c_double],
    "mdlj_features": [_ctxp, C.POINTER(C.c_float)],
    "mdlj_mlp_load": [_ctxp, C.c_char_p],
    "mdlj_mlp_save": [_ctxp, C.c_char_p],
    "mdlj_mlp_set_threshold": [_ctxp, C.c_double],
    "mdlj_set_timing": [_ctxp, C.c_int32],
    "mdlj_mlp_init": [_ctxp, C.c_int32, C.c_uint64],
    "mdlj_mlp_set_norm": [_ctxp, C.POINTER(C.c_float), C.POINTER(C.c_float)],
    "mdlj_mlp_get_params": [_ctxp, C.POINTER(C.c_float), C.c_int64, C.POINTER(C.c_int64),
                            C.POINTER(C.c_int32)],
    "mdlj_mlp_set_params": [_ctxp, C.POINTER(C.c_float), C.c_int64, C.c_int32],
    "mdlj_mlp_predict": [_ctxp, C.POINTER(C.c_float), C.c_int32, C.POINTER(C.c_float)],
    "mdlj_mlp_loss_grad": [_ctxp, C.POINTER(C.c_float), C.POINTER(C.c_int32), C.c_int32,
                           C.POINTER(C.c_float), C.POINTER(C.c_float)],
    "mdlj_mlp_train": [_ctxp, C.POINTER(C.c_float), C.POINTER(C.c_int32), C.c_int32, C.c_int32,
                       C.c_int32, C.c_double, C.c_uint64, C.POINTER(C.c_double)],
    "mdlj_mlp_stats": [_ctxp, C.POINTER(C.c_double), C.POINTER(C.c_int64)],
    "mdlj_tune_select": [_d, C.c_int32, C.c_int32, C.c_int32, _d, C.POINTER(C.c_int32)],
    "mdlj_retune_needed": [C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_double,
                           C.POINTER(C.c_int32)],
    "mdlj_get_timing": [_ctxp, _d, _d, C.POINTER(C.c_int64), C.POINTER(C.c_int64)],
    "mdlj_get_timing_fused": [_ctxp, _d, C.POINTER(C.c_int64)],
    "mdlj_set_tune_metric": [_ctxp, C.c_int32],
    "mdlj_lane_map": [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.POINTER(C.c_int32),
                      C.POINTER(C.c_int32)],
    "mdlj_config_lane_map": [C.POINTER(mdlj_config), C.c_int32, C.POINTER(C.c_int32),
                             C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
    "mdlj_tune_power": [_ctxp, _d, C.c_int32, C.POINTER(C.c_int32)],
    "mdlj_gpu_energy": [_ctxp, _d, _d],
    "mdlj_tune_select_energy": [_d, _d, C.c_int32, _d, C.POINTER(C.c_int32)],
    "mdlj_compute_forces_noalloc": [_ctxp, _vp, _vp, _vp, _d, _d],
    "mdlj_get_cells": [_ctxp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)],
    "mdlj_get_pairs": [_ctxp, C.c_int64, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                       C.POINTER(C.c_int64)],
}
for _name, _args in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = C.c_int
lib.mdlj_last_error.argtypes = [_ctxp]
lib.mdlj_last_error.restype = C.c_char_p
lib.mdlj_version.argtypes = []
lib.mdlj_version.restype = C.c_char_p


def last_error(ctx) -> str:
    m = lib.mdlj_last_error(ctx)
    return m.decode() if m else ""


def check(status, ctx=None):
    if status != MDLJ_OK:
        raise MdljError(status, last_error(ctx) if ctx else "")
    return status


# names of the C ABI, callable directly -----------------------------------
def __getattr__(name):
    if name.startswith("mdlj_"):
        return getattr(lib, name)
    raise AttributeError(name)


def _ptr(a):
    """(pointer, mem_kind) of a torch tensor or NumPy array."""
    if hasattr(a, "data_ptr"):
        if a.is_cuda:
            return C.c_void_p(a.data_ptr()), MEM_DEVICE
        return C.c_void_p(a.data_ptr()), MEM_HOST
    return a.ctypes.data_as(C.c_void_p), MEM_HOST


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class System:
    """Owns one mdlj context.  pos: (n, 3) float64 NumPy array or torch CUDA
    tensor; types: int32 per particle or None."""

    def __init__(self, pos, box, rc, eps=(1.0,), sig=(1.0,), types=None, skin=0.0,
                 rebuild_every=10, shift=True, precision=PREC_F32PAIR_F64ACC, stream=None,
                 mass=None):
        eps = list(np.atleast_1d(eps))
        sig = list(np.atleast_1d(sig))
        nspec = len(eps)
        self._keep = []
        n = int(pos.shape[0])
        cols = self._cols(pos)
        tptr = None
        if types is not None:
            if hasattr(types, "data_ptr"):
                tt = types.to(dtype=__import__("torch").int32).contiguous()
            else:
                tt = np.ascontiguousarray(types, dtype=np.int32)
            self._keep.append(tt)
            tptr, tk = _ptr(tt)
        px, kind = _ptr(cols[0])
        py, _ = _ptr(cols[1])
        pz, _ = _ptr(cols[2])
        if tptr is not None and tk != kind:
            raise ValueError("positions and types must live in the same memory")
        h = _ctxp()
        check(lib.mdlj_create(C.byref(h), n, px, py, pz, tptr, nspec, kind,
                              _stream_handle(stream)))
        self.ctx = h
        self.n = n
        self.nspec = nspec
        self.box = np.asarray(box, np.float64)
        try:
            check(lib.mdlj_set_box(h, *map(float, self.box)), h)
            check(lib.mdlj_set_cutoff(h, float(rc)), h)
            check(lib.mdlj_set_skin(h, float(skin), int(rebuild_every)), h)
            for s in range(nspec):
                check(lib.mdlj_set_species(h, s, float(eps[s]), float(sig[s])), h)
                if mass is not None:
                    check(lib.mdlj_set_mass(h, s, float(np.atleast_1d(mass)[s])), h)
            check(lib.mdlj_set_energy_shift(h, int(bool(shift))), h)
            check(lib.mdlj_set_precision(h, int(precision)), h)
        except Exception:
            self.close()
            raise

    @staticmethod
    def _cols(pos):
        if hasattr(pos, "data_ptr"):
            return [pos[:, k].contiguous() for k in range(3)]
        pos = np.asarray(pos, np.float64)
        return [np.ascontiguousarray(pos[:, k]) for k in range(3)]

    def close(self):
        if getattr(self, "ctx", None):
            lib.mdlj_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        self.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    # --- configuration --------------------------------------------------
    def configs(self):
        n = C.c_int32()
        check(lib.mdlj_config_count(self.ctx, C.byref(n)), self.ctx)
        out = []
        for k in range(n.value):
            c = mdlj_config()
            check(lib.mdlj_config_at(self.ctx, k, C.byref(c)), self.ctx)
            out.append(c)
        return out

    def set_config(self, cfg):
        if not isinstance(cfg, mdlj_config):
            cfg = mdlj_config(*cfg)
        check(lib.mdlj_set_config(self.ctx, C.byref(cfg)), self.ctx)

    def get_config(self):
        c = mdlj_config()
        check(lib.mdlj_get_config(self.ctx, C.byref(c)), self.ctx)
        return c

    def set_precision(self, prec):
        check(lib.mdlj_set_precision(self.ctx, int(prec)), self.ctx)

    # --- state ------------------------------------------------------------
    def set_positions(self, pos):
        cols = self._cols(pos)
        px, kind = _ptr(cols[0])
        py, _ = _ptr(cols[1])
        pz, _ = _ptr(cols[2])
        check(lib.mdlj_set_positions(self.ctx, px, py, pz, kind), self.ctx)

    def get_positions(self):
        out = [np.empty(self.n) for _ in range(3)]
        check(lib.mdlj_get_positions(self.ctx, *[_ptr(o)[0] for o in out], MEM_HOST), self.ctx)
        return np.stack(out, 1)

    def rebuild(self):
        check(lib.mdlj_rebuild_neighbors(self.ctx), self.ctx)

    def forces(self, out=None, energy=True):
        """Forces (n, 3) in caller order plus (U, W).  out: optional tuple of
        three device tensors (or host arrays) to fill."""
        if out is None:
            out = [np.empty(self.n) for _ in range(3)]
        ptrs = [_ptr(o) for o in out]
        U = C.c_double()
        W = C.c_double()
        check(lib.mdlj_compute_forces(self.ctx, ptrs[0][0], ptrs[1][0], ptrs[2][0],
                                      ptrs[0][1], C.byref(U) if energy else None,
                                      C.byref(W) if energy else None), self.ctx)
        if isinstance(out[0], np.ndarray):
            f = np.stack(out, 1)
        else:
            f = out
        return f, U.value, W.value

    def forces_noalloc(self, out, energy=True):
        """mdlj_compute_forces_noalloc into three device tensors; returns
        (out, U, W)."""
        ptrs = [_ptr(o) for o in out]
        if any(k != MEM_DEVICE for _, k in ptrs):
            raise ValueError("outputs must be device tensors")
        U = C.c_double()
        W = C.c_double()
        check(lib.mdlj_compute_forces_noalloc(self.ctx, ptrs[0][0], ptrs[1][0], ptrs[2][0],
                                              C.byref(U) if energy else None,
                                              C.byref(W) if energy else None), self.ctx)
        return out, U.value, W.value

    def neighbor_stats(self):
        """(stored list entries incl. row padding, bytes per entry, records)."""
        e, r = C.c_int64(), C.c_int64()
        b = C.c_int32()
        check(lib.mdlj_neighbor_stats(self.ctx, C.byref(e), C.byref(b), C.byref(r)), self.ctx)
        return e.value, b.value, r.value

    def get_cells(self):
        """(cell of every particle in the last binning, x-fastest over the
        interior grid; grid cell counts (nx, ny, nz))."""
        cell = np.empty(self.n, np.int32)
        nc = np.empty(3, np.int32)
        i32 = C.POINTER(C.c_int32)
        check(lib.mdlj_get_cells(self.ctx, cell.ctypes.data_as(i32), nc.ctypes.data_as(i32)),
              self.ctx)
        return cell, tuple(int(v) for v in nc)

    def get_pairs(self):
        """(pi, pj) caller indices of the pairs the current list holds."""
        cnt = C.c_int64()
        check(lib.mdlj_get_pairs(self.ctx, 0, None, None, C.byref(cnt)), self.ctx)
        pi = np.empty(cnt.value, np.int32)
        pj = np.empty(cnt.value, np.int32)
        i32 = C.POINTER(C.c_int32)
        check(lib.mdlj_get_pairs(self.ctx, cnt.value, pi.ctypes.data_as(i32),
                                 pj.ctypes.data_as(i32), C.byref(cnt)), self.ctx)
        return pi[: cnt.value], pj[: cnt.value]

    def count_pairs(self):
        n = C.c_int64()
        check(lib.mdlj_count_pairs(self.ctx, C.byref(n)), self.ctx)
        return n.value

    def tune(self, mode=TUNE_EXHAUSTIVE, samples=10):
        c = mdlj_config()
        us = C.c_double()
        check(lib.mdlj_tune(self.ctx, int(mode), int(samples), C.byref(c), C.byref(us)),
              self.ctx)
        return c, us.value

    def tune_results(self):
        n = C.c_int32()
        buf = (C.c_double * 256)()
        check(lib.mdlj_tune_results(self.ctx, buf, 256, C.byref(n)), self.ctx)
        return np.array(buf[: n.value])

    def set_pruning(self, on):
        check(lib.mdlj_set_pruning(self.ctx, int(bool(on))), self.ctx)

    def pruning_state(self, tiles=False):
        """0 no inner list, 1 valid everywhere, 2 given up in some tiles, 3
        given up everywhere; with tiles=True also the count of tiles that gave
        it up."""
        v = C.c_int32()
        t = C.c_int64()
        check(lib.mdlj_pruning_state(self.ctx, C.byref(v), C.byref(t)), self.ctx)
        return (v.value, t.value) if tiles else v.value

    def set_tune_metric(self, metric):
        check(lib.mdlj_set_tune_metric(self.ctx, int(metric)), self.ctx)

    def tune_power(self):
        n = C.c_int32()
        buf = (C.c_double * 256)()
        check(lib.mdlj_tune_power(self.ctx, buf, 256, C.byref(n)), self.ctx)
        return np.array(buf[: n.value])

    def gpu_energy(self):
        """(joules, seconds) of the GPU's energy counter and its last refresh."""
        j, s = C.c_double(), C.c_double()
        check(lib.mdlj_gpu_energy(self.ctx, C.byref(j), C.byref(s)), self.ctx)
        return j.value, s.value

    def tune_taken(self):
        n = C.c_int32()
        buf = (C.c_int32 * 256)()
        check(lib.mdlj_tune_taken(self.ctx, buf, 256, C.byref(n)), self.ctx)
        return np.array(buf[: n.value])

    def step_vv(self, vel_cols, dt, nsteps):
        ptrs = [_ptr(v) for v in vel_cols]
        if any(k != MEM_DEVICE for _, k in ptrs):
            raise ValueError("velocities must be device tensors")
        check(lib.mdlj_step_vv(self.ctx, ptrs[0][0], ptrs[1][0], ptrs[2][0], float(dt),
                               int(nsteps)), self.ctx)

    def set_timing(self, on=True):
        check(lib.mdlj_set_timing(self.ctx, int(bool(on))), self.ctx)

    def get_timing(self):
        """(force_us_total, build_us_total, n_force, n_build) since set_timing."""
        f, b = C.c_double(), C.c_double()
        nf, nb = C.c_int64(), C.c_int64()
        check(lib.mdlj_get_timing(self.ctx, C.byref(f), C.byref(b), C.byref(nf), C.byref(nb)),
              self.ctx)
        return f.value, b.value, nf.value, nb.value

    def get_timing_fused(self):
        """(us_total, n) of the timed force kernels that took the integrator
        step too, since set_timing."""
        f, nf = C.c_double(), C.c_int64()
        check(lib.mdlj_get_timing_fused(self.ctx, C.byref(f), C.byref(nf)), self.ctx)
        return f.value, nf.value

    # --- learned tuner network -------------------------------------------
    def mlp_init(self, k, seed=0):
        check(lib.mdlj_mlp_init(self.ctx, int(k), int(seed)), self.ctx)

    def mlp_set_norm(self, mean, std):
        mean = np.ascontiguousarray(mean, np.float32)
        std = np.ascontiguousarray(std, np.float32)
        check(lib.mdlj_mlp_set_norm(self.ctx, _fp(mean), _fp(std)), self.ctx)

    def mlp_params(self):
        n = C.c_int64()
        k = C.c_int32()
        check(lib.mdlj_mlp_get_params(self.ctx, None, 0, C.byref(n), C.byref(k)), self.ctx)
        w = np.empty(n.value, np.float32)
        check(lib.mdlj_mlp_get_params(self.ctx, _fp(w), n.value, C.byref(n), C.byref(k)),
              self.ctx)
        return w, k.value

    def mlp_set_params(self, w, k):
        w = np.ascontiguousarray(w, np.float32)
        check(lib.mdlj_mlp_set_params(self.ctx, _fp(w), w.size, int(k)), self.ctx)

    def mlp_predict(self, X):
        X = np.ascontiguousarray(np.atleast_2d(X), np.float32)
        _, k = self.mlp_params()
        out = np.empty((len(X), k), np.float32)
        check(lib.mdlj_mlp_predict(self.ctx, _fp(X), len(X), _fp(out)), self.ctx)
        return out

    def mlp_loss_grad(self, X, y):
        X = np.ascontiguousarray(np.atleast_2d(X), np.float32)
        y = np.ascontiguousarray(y, np.int32)
        w, _ = self.mlp_params()
        g = np.empty_like(w)
        loss = C.c_float()
        check(lib.mdlj_mlp_loss_grad(self.ctx, _fp(X), y.ctypes.data_as(C.POINTER(C.c_int32)),
                                     len(X), _fp(g), C.byref(loss)), self.ctx)
        return loss.value, g

    def mlp_train(self, X, y, epochs, batch=64, lr=1e-3, seed=0):
        X = np.ascontiguousarray(np.atleast_2d(X), np.float32)
        y = np.ascontiguousarray(y, np.int32)
        loss = C.c_double()
        check(lib.mdlj_mlp_train(self.ctx, _fp(X), y.ctypes.data_as(C.POINTER(C.c_int32)),
                                 len(X), int(epochs), int(batch), float(lr), int(seed),
                                 C.byref(loss)), self.ctx)
        return loss.value

    def mlp_load(self, path):
        check(lib.mdlj_mlp_load(self.ctx, str(path).encode()), self.ctx)

    def mlp_save(self, path):
        check(lib.mdlj_mlp_save(self.ctx, str(path).encode()), self.ctx)

    def mlp_set_threshold(self, t):
        check(lib.mdlj_mlp_set_threshold(self.ctx, float(t)), self.ctx)

    def mlp_stats(self):
        c = C.c_double()
        f = C.c_int64()
        check(lib.mdlj_mlp_stats(self.ctx, C.byref(c), C.byref(f)), self.ctx)
        return c.value, f.value

    def features(self):
        f = (C.c_float * 8)()
        check(lib.mdlj_features(self.ctx, f), self.ctx)
        return np.array(f[:], np.float32)


def tune_select(samples, mode=0):
    """Reduced value per configuration and the chosen index for a [K, S]
    table of timings (the full-search decision rule of the tuner)."""
    a = np.ascontiguousarray(np.atleast_2d(samples), np.float64)
    vals = np.empty(a.shape[0])
    ch = C.c_int32()
    check(lib.mdlj_tune_select(a.ctypes.data_as(_d), a.shape[0], a.shape[1], int(mode),
                               vals.ctypes.data_as(_d), C.byref(ch)))
    return vals, ch.value


def tune_select_early(samples, order=None, warm_factor=2.0, margin=0.1):
    """The early-stopping search over a [K, S] table (sample 0 = warm-up):
    (values, samples taken, chosen index)."""
    a = np.ascontiguousarray(np.atleast_2d(samples), np.float64)
    k, s = a.shape
    vals = np.empty(k)
    taken = np.empty(k, np.int32)
    ch = C.c_int32()
    i32 = C.POINTER(C.c_int32)
    o = None if order is None else np.ascontiguousarray(order, np.int32)
    check(lib.mdlj_tune_select_early(a.ctypes.data_as(_d), k, s,
                                     None if o is None else o.ctypes.data_as(i32),
                                     float(warm_factor), float(margin), vals.ctypes.data_as(_d),
                                     taken.ctypes.data_as(i32), C.byref(ch)))
    return vals, taken, ch.value


def lane_map(layout, ai, width):
    """(i offsets, j offsets) of the lanes of one step: layout 0 j fastest,
    1 i fastest, ai i's in a vector of width lanes."""
    i, j = C.c_int32(), C.c_int32()
    out = []
    for lane in range(width):
        check(lib.mdlj_lane_map(int(layout), int(ai), int(width), lane, C.byref(i), C.byref(j)))
        out.append((i.value, j.value))
    return np.array(out, np.int32).T


def config_lane_map(cfg):
    """(layout, i offsets, j offsets) of the 64 lanes of one step of a
    configuration's kernel."""
    if not isinstance(cfg, mdlj_config):
        cfg = mdlj_config(*cfg)
    lay, i, j = C.c_int32(), C.c_int32(), C.c_int32()
    out = []
    for lane in range(64):
        check(lib.mdlj_config_lane_map(C.byref(cfg), lane, C.byref(lay), C.byref(i), C.byref(j)))
        out.append((i.value, j.value))
    a = np.array(out, np.int32).T
    return lay.value, a[0], a[1]


def tune_select_energy(us, watts):
    """Energy per step (microjoules) of each configuration and the chosen index."""
    u = np.ascontiguousarray(us, np.float64)
    w = np.ascontiguousarray(watts, np.float64)
    out = np.empty(len(u))
    ch = C.c_int32()
    check(lib.mdlj_tune_select_energy(u.ctypes.data_as(_d), w.ctypes.data_as(_d), len(u),
                                      out.ctypes.data_as(_d), C.byref(ch)))
    return out, ch.value


def retune_needed(before, now, threshold=0.1):
    b = np.ascontiguousarray(before, np.float32)
    n = np.ascontiguousarray(now, np.float32)
    out = C.c_int32()
    check(lib.mdlj_retune_needed(_fp(b), _fp(n), float(threshold), C.byref(out)))
    return bool(out.value)


def version() -> str:
    return lib.mdlj_version().decode()
