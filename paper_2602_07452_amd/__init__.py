"""Python binding of the MI355X GRPIC library (``libgrpic.so``, include/grpic.h).

Argument marshalling only: every step of the method runs in the HIP kernels
of the library.  The binding refuses to work without the built library (there
is no CPU fallback).  Names follow the C ABI without the ``grpic_`` prefix.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GRPIC_LIBRARY") or os.path.join(_HERE, "libgrpic.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "grpic.h")
_LIB = None

# enums (include/grpic.h)
PUSH_RK4, PUSH_IMR, PUSH_HAM, PUSH_HYB1, PUSH_HYB2 = 0, 1, 2, 3, 4
GUESS_PLAIN, GUESS_RK4, GUESS_MLP = 0, 1, 2
FIELDS_NONE, FIELDS_STATIC, FIELDS_EVOLVE = 0, 1, 2
LEVEL_DN, LEVEL_DH0, LEVEL_DH1, LEVEL_BM, LEVEL_BN, LEVEL_BH, LEVEL_J, LEVEL_JPREV = range(8)
INIT_ORBITS, INIT_SHELL_ISO, INIT_SHELL_MJ = 0, 1, 2
FLAG_ALIVE, FLAG_IMPLICIT, FLAG_NOCONV, FLAG_REMOVED, FLAG_REFLECTED = 1, 2, 4, 8, 16
FLAG_NONFINITE = 32
K_FIELDS, K_PUSH, K_IMPLICIT, K_DEPOSIT, K_SORT, K_GUESS, K_CLEAN = range(7)
KERNEL_NAMES = ("fields", "push", "implicit", "deposit", "sort", "guess", "clean")
DEPOSIT_CONSERVING, DEPOSIT_PAPER = 0, 1
SOLVER_PICARD, SOLVER_NEWTON = 0, 1
HIST_BINS = 64
MLP_NPARAM = 5510


class GrpicError(RuntimeError):
    pass


class Config(C.Structure):
    _fields_ = [("a", C.c_double), ("nr", C.c_int), ("nth", C.c_int),
                ("r_in", C.c_double), ("r_out", C.c_double), ("theta0", C.c_double),
                ("dt", C.c_double), ("field_mode", C.c_int), ("pusher", C.c_int),
                ("guess", C.c_int), ("hyb_threshold", C.c_double), ("tol", C.c_double),
                ("kmax", C.c_int), ("ham_eps", C.c_double), ("r_abs", C.c_double),
                ("chi0", C.c_double), ("lambda_abs", C.c_double),
                ("r_remove_in", C.c_double), ("r_remove_out", C.c_double),
                ("reflect", C.c_int), ("max_particles", C.c_long),
                ("sort_every", C.c_int), ("tile_r", C.c_int), ("tile_th", C.c_int),
                ("block", C.c_int), ("persistent_waves", C.c_int),
                ("push_waves_per_simd", C.c_int), ("dt_implicit", C.c_double),
                ("t_end", C.c_double), ("deposit_mode", C.c_int), ("clean_every", C.c_int),
                ("clean_iters", C.c_int), ("inj_every", C.c_int), ("inj_r0", C.c_double),
                ("inj_r1", C.c_double), ("inj_mult", C.c_double), ("inj_density", C.c_double),
                ("inj_theta", C.c_double), ("inj_seed", C.c_uint64), ("solver", C.c_int)]


class InitSpec(C.Structure):
    _fields_ = [("kind", C.c_int), ("n", C.c_long), ("seed", C.c_uint64),
                ("r0", C.c_double), ("r1", C.c_double), ("t0", C.c_double),
                ("t1", C.c_double), ("p0", C.c_double), ("w", C.c_double)]


class Diag(C.Structure):
    _fields_ = [("steps", C.c_long), ("alive", C.c_long), ("removed", C.c_long),
                ("implicit_steps", C.c_long), ("noconv", C.c_long),
                ("reflected", C.c_long), ("iter_hist", C.c_long * HIST_BINS),
                ("herr_hist", C.c_long * HIST_BINS), ("deposit_fallback", C.c_long),
                ("nonfinite", C.c_long), ("deposit_outside", C.c_long)]


def lib():
    """Load libgrpic.so (built by ``__graft_entry__.build()``)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise GrpicError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        L.grpic_last_error.restype = C.c_char_p
        L.grpic_last_error.argtypes = [C.c_void_p]
        L.grpic_create.argtypes = [C.POINTER(Config), C.POINTER(C.c_void_p)]
        L.grpic_destroy.argtypes = [C.c_void_p]
        L.grpic_destroy.restype = None
        _LIB = L
    return _LIB


def exported_symbols():
    """Names of the functions declared in include/grpic.h."""
    with open(HEADER) as f:
        txt = f.read()
    return sorted(set(re.findall(r"\b(grpic_[a-z_0-9]+)\s*\(", txt)))


def _check(rc, ctx=None):
    if rc != 0:
        msg = lib().grpic_last_error(ctx)
        raise GrpicError(f"grpic error {rc}: {msg.decode() if msg else ''}")


def config_default(**kw) -> Config:
    cfg = Config()
    _check(lib().grpic_config_default(C.byref(cfg)))
    for k, v in kw.items():
        if not hasattr(cfg, k):
            raise KeyError(k)
        setattr(cfg, k, v)
    return cfg


def cfl_dt(cfg: Config) -> float:
    out = C.c_double()
    _check(lib().grpic_cfl_dt(C.byref(cfg), C.byref(out)))
    return out.value


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


class Context:
    """One GRPIC simulation context on the current HIP device."""

    def __init__(self, cfg: Config):
        h = C.c_void_p()
        _check(lib().grpic_create(C.byref(cfg), C.byref(h)))
        self._h = h
        self.cfg = self.get_config()  # dt resolved (0: half the Courant limit)

    def get_config(self) -> Config:
        """The configuration as the library holds it now."""
        out = Config()
        self._c("grpic_get_config", C.byref(out))
        return out

    # -- lifetime
    def close(self):
        if getattr(self, "_h", None):
            lib().grpic_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _c(self, fn, *args):
        _check(getattr(lib(), fn)(self._h, *args), self._h)

    # -- streams
    def set_stream(self, stream_handle: int | None):
        self._c("grpic_set_stream", C.c_void_p(stream_handle or 0))

    def sync(self):
        self._c("grpic_sync")

    # -- grid
    def grid_coords(self):
        nr, nth = self.cfg.nr, self.cfg.nth
        rn, rh, tn, th = np.zeros(nr + 1), np.zeros(nr), np.zeros(nth + 1), np.zeros(nth)
        self._c("grpic_grid_coords", _dp(rn), _dp(rh), _dp(tn), _dp(th))
        return rn, rh, tn, th

    def field_shape(self, level, comp):
        """(rows = theta, cols = r) of a densitized component."""
        nr, nth = self.cfg.nr, self.cfg.nth
        if LEVEL_BM <= level <= LEVEL_BH:
            rh, thh = comp in (1, 2), comp in (0, 2)
        else:
            rh, thh = comp == 0, comp == 1
        return (nth if thh else nth + 1, nr if rh else nr + 1)

    def set_fields_wald(self, B0, a_field=None):
        """Wald field; a_field (default: the spacetime spin) is the spin in
        the potential, 0 for the Schwarzschild-Wald start."""
        af = self.cfg.a if a_field is None else a_field
        self._c("grpic_set_fields_wald", C.c_double(B0), C.c_double(af))

    def set_fields_split_monopole(self, B0, zeta0):
        self._c("grpic_set_fields_split_monopole", C.c_double(B0), C.c_double(zeta0))

    def set_field(self, level, comp, arr):
        a = np.ascontiguousarray(arr, dtype=np.float32)
        if a.shape != self.field_shape(level, comp):
            raise ValueError(f"shape {a.shape} != {self.field_shape(level, comp)}")
        self._c("grpic_set_field", level, comp, a.ctypes.data_as(C.POINTER(C.c_float)))

    def get_field(self, level, comp):
        a = np.zeros(self.field_shape(level, comp), dtype=np.float32)
        self._c("grpic_get_field", level, comp, a.ctypes.data_as(C.POINTER(C.c_float)))
        return a

    # -- particles
    def init_particles(self, kind, n, seed, r0, r1, t0, t1, p0, w=1.0):
        spec = InitSpec(kind, n, seed, r0, r1, t0, t1, p0, w)
        self._c("grpic_init_particles", C.byref(spec))

    def load_particles(self, z, qm, w=None, H0=None, herr=None):
        z = np.atleast_2d(_f64(z))
        n = z.shape[0]
        cols = [np.ascontiguousarray(z[:, i]) for i in range(6)]
        qm = _f64(np.broadcast_to(qm, (n,)))
        w = _f64(np.ones(n) if w is None else np.broadcast_to(w, (n,)))
        H0a = None if H0 is None else _f64(H0)
        herra = None if herr is None else _f64(herr)
        H0p = _dp(H0a) if H0a is not None else None
        hp = _dp(herra) if herra is not None else None
        self._c("grpic_load_particles", C.c_long(n), *[_dp(c) for c in cols],
                _dp(qm), _dp(w), H0p, hp)

    def num_particles(self):
        n = C.c_long()
        self._c("grpic_num_particles", C.byref(n))
        return n.value

    def get_particles(self):
        n = self.num_particles()
        out = {k: np.zeros(n) for k in ("r", "th", "ph", "ur", "uth", "uph", "qm", "w",
                                         "H0", "herr")}
        flags = np.zeros(n, np.int32)
        iters = np.zeros(n, np.int32)
        ip = C.POINTER(C.c_int32)
        self._c("grpic_get_particles", C.c_long(n),
                *[_dp(out[k]) for k in ("r", "th", "ph", "ur", "uth", "uph", "qm", "w",
                                         "H0", "herr")],
                flags.ctypes.data_as(ip), iters.ctypes.data_as(ip))
        out["flags"], out["iters"] = flags, iters
        out["z"] = np.stack([out[k] for k in ("r", "th", "ph", "ur", "uth", "uph")], axis=1)
        return out

    def get_times(self):
        """Each particle's own time (no grid), in id order."""
        n = self.num_particles()
        t = np.zeros(n)
        self._c("grpic_get_times", C.c_long(n), _dp(t))
        return t

    def sample_particles(self, ids):
        """Particle records of the given ids, as get_particles() returns them."""
        ids = np.ascontiguousarray(ids, dtype=np.int64)
        m = len(ids)
        rec = np.zeros((m, 10))
        flags = np.zeros(m, np.int32)
        iters = np.zeros(m, np.int32)
        ip = C.POINTER(C.c_int32)
        self._c("grpic_sample_particles", C.c_long(m), ids.ctypes.data_as(C.POINTER(C.c_long)),
                _dp(rec), flags.ctypes.data_as(ip), iters.ctypes.data_as(ip))
        out = {k: np.ascontiguousarray(rec[:, i]) for i, k in enumerate(
            ("r", "th", "ph", "ur", "uth", "uph", "qm", "w", "H0", "herr"))}
        out["flags"], out["iters"] = flags, iters
        out["z"] = rec[:, :6].copy()
        return out

    # -- snapshots
    def get_state(self):
        """The context's snapshot (header, fields, particles, counters) as a
        uint8 array."""
        nb = C.c_size_t()
        self._c("grpic_state_size", C.byref(nb))
        buf = np.zeros(nb.value, np.uint8)
        self._c("grpic_get_state", buf.ctypes.data_as(C.c_void_p), C.c_size_t(nb.value))
        return buf

    def set_state(self, buf):
        """Restore a snapshot taken by get_state() (same grid, mode, dt)."""
        buf = np.ascontiguousarray(np.frombuffer(buf, np.uint8))
        self._c("grpic_set_state", buf.ctypes.data_as(C.c_void_p), C.c_size_t(buf.size))

    # -- stepping
    def step(self, nsteps=1):
        self._c("grpic_step", C.c_int(nsteps))

    def use_graph(self, enable=True):
        self._c("grpic_use_graph", C.c_int(1 if enable else 0))

    # -- diagnostics
    def diagnostics(self):
        d = Diag()
        self._c("grpic_get_diagnostics", C.byref(d))
        return {"steps": d.steps, "alive": d.alive, "removed": d.removed,
                "implicit_steps": d.implicit_steps, "noconv": d.noconv,
                "reflected": d.reflected, "iter_hist": np.array(d.iter_hist[:]),
                "herr_hist": np.array(d.herr_hist[:]),
                "deposit_fallback": d.deposit_fallback, "nonfinite": d.nonfinite,
                "deposit_outside": d.deposit_outside}

    def inject(self):
        """Pair injection now (Sec. 3.3); returns the particles added."""
        n = C.c_long()
        self._c("grpic_inject", C.byref(n))
        return n.value

    def clean(self, iters=500):
        """Divergence cleaning of both D chains now (Sec. 2.4)."""
        self._c("grpic_clean", C.c_int(iters))

    def field_diagnostics(self):
        g, b = C.c_double(), C.c_double()
        p = np.zeros(self.cfg.nr + 1)
        self._c("grpic_field_diagnostics", C.byref(g), C.byref(b), _dp(p))
        return g.value, b.value, p

    def field_diagnostics_noalloc(self):
        g, b = C.c_double(), C.c_double()
        p = np.zeros(self.cfg.nr + 1)
        self._c("grpic_field_diagnostics_noalloc", C.byref(g), C.byref(b), _dp(p))
        return g.value, b.value, p

    # -- timing
    def enable_timing(self, enable=True):
        self._c("grpic_enable_timing", C.c_int(1 if enable else 0))

    def reset_timings(self):
        self._c("grpic_reset_timings")

    def timings(self):
        k = len(KERNEL_NAMES)  # GRPIC_K_COUNT
        ms = np.zeros(k)
        cnt = np.zeros(k, dtype=np.int64)
        self._c("grpic_get_timings", _dp(ms), cnt.ctypes.data_as(C.POINTER(C.c_long)))
        return {KERNEL_NAMES[i]: (float(ms[i]), int(cnt[i])) for i in range(k)}

    # -- learned guess
    def mlp_set(self, theta, mean, inv_std, scale):
        keep = [np.ascontiguousarray(x, dtype=np.float32) for x in (theta, mean, inv_std, scale)]
        assert keep[0].size == MLP_NPARAM and keep[1].size == 14 and keep[3].size == 6
        self._c("grpic_mlp_set", *[k.ctypes.data_as(C.POINTER(C.c_float)) for k in keep])

    # -- autotuner
    def autotune(self, trial_steps=3):
        r = TuneResult()
        self._c("grpic_autotune", C.c_int(trial_steps), C.byref(r))
        self.cfg.tile_r, self.cfg.tile_th = r.tile_r, r.tile_th
        self.cfg.persistent_waves = r.persistent_waves
        self.cfg.push_waves_per_simd = r.push_waves_per_simd
        return {f[0]: getattr(r, f[0]) for f in TuneResult._fields_}

    def probe_peaks(self):
        """Measured FP64 FMA rate (TFLOP/s) and streaming copy rate (TB/s) of
        the context's device."""
        f, b = C.c_double(), C.c_double()
        self._c("grpic_probe_peaks", C.byref(f), C.byref(b))
        return {"fp64_fma_tflops": f.value, "copy_tbs": b.value}

    def mlp_get(self):
        theta = np.zeros(MLP_NPARAM, np.float32)
        mean, inv_std, scale = np.zeros(14, np.float32), np.zeros(14, np.float32), np.zeros(6, np.float32)
        fp = C.POINTER(C.c_float)
        self._c("grpic_mlp_get", *[x.ctypes.data_as(fp) for x in (theta, mean, inv_std, scale)])
        return theta, mean, inv_std, scale

    def mlp_collect(self, max_rows):
        self._c("grpic_mlp_collect", C.c_long(max_rows))

    def mlp_num_samples(self):
        n = C.c_long()
        self._c("grpic_mlp_num_samples", C.byref(n))
        return n.value

    def mlp_get_samples(self, n=None):
        n = self.mlp_num_samples() if n is None else n
        X = np.zeros((n, 14), np.float32)
        T = np.zeros((n, 6), np.float32)
        valid = np.zeros(n, np.uint8)
        fp = C.POINTER(C.c_float)
        self._c("grpic_mlp_get_samples", C.c_long(n), X.ctypes.data_as(fp),
                T.ctypes.data_as(fp), valid.ctypes.data_as(C.POINTER(C.c_ubyte)))
        return X, T, valid

    def mlp_train(self, epochs=8, batch=16384, lr=2e-3, lr_final=2e-5, beta1=0.9,
                  beta2=0.999, eps=1e-8, seed=1):
        tc = MlpTrainConfig(epochs, batch, lr, lr_final, beta1, beta2, eps, seed)
        loss = np.zeros(epochs)
        self._c("grpic_mlp_train", C.byref(tc), _dp(loss))
        return loss

    def mlp_forward(self, X):
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, 14)
        Y = np.zeros((X.shape[0], 6), np.float32)
        fp = C.POINTER(C.c_float)
        self._c("grpic_mlp_forward", C.c_long(X.shape[0]), X.ctypes.data_as(fp),
                Y.ctypes.data_as(fp))
        return Y

    def mlp_loss_grad(self, X, T):
        X = np.ascontiguousarray(X, dtype=np.float32).reshape(-1, 14)
        T = np.ascontiguousarray(T, dtype=np.float32).reshape(-1, 6)
        g = np.zeros(MLP_NPARAM, np.float32)
        loss = C.c_double()
        fp = C.POINTER(C.c_float)
        self._c("grpic_mlp_loss_grad", C.c_long(X.shape[0]), X.ctypes.data_as(fp),
                T.ctypes.data_as(fp), g.ctypes.data_as(fp), C.byref(loss))
        return loss.value, g


class StateHeader(C.Structure):
    _fields_ = [("magic", C.c_char * 8), ("version", C.c_int32), ("field_mode", C.c_int32),
                ("nr", C.c_int32), ("nth", C.c_int32), ("a", C.c_double), ("r_in", C.c_double),
                ("r_out", C.c_double), ("theta0", C.c_double), ("dt", C.c_double),
                ("n", C.c_int64), ("steps", C.c_int64), ("qw_max", C.c_double),
                ("has_neutral", C.c_int32), ("reserved", C.c_int32), ("bytes", C.c_uint64)]


def state_header(buf):
    """The header of a snapshot block."""
    return StateHeader.from_buffer_copy(bytes(np.asarray(buf, np.uint8)[:C.sizeof(StateHeader)]))


class TuneResult(C.Structure):
    _fields_ = [("tile_r", C.c_int), ("tile_th", C.c_int), ("persistent_waves", C.c_int),
                ("push_waves_per_simd", C.c_int), ("trials", C.c_int), ("steps", C.c_int),
                ("ms_start", C.c_double), ("ms_best", C.c_double)]


class MlpTrainConfig(C.Structure):
    _fields_ = [("epochs", C.c_long), ("batch", C.c_long), ("lr", C.c_double),
                ("lr_final", C.c_double), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("seed", C.c_uint64)]
