"""Reference oracle for the GRPIC particle hot path (TEST INFRASTRUCTURE).

Plain FP64 CPU implementation of arXiv:2602.07452's method written from the
paper (C in ``om_*.c``, bound here with ctypes).  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import this package; the
GPU library never calls it and shares no code with it.

Field arrays are NumPy float64, r-fastest, shaped (nT, nR) for the component's
staggered sub-grid (see ``grpic_oracle.h`` for the Yee layout).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

D_P = C.POINTER(C.c_double)
I_P = C.POINTER(C.c_int)

RK4, IMR, HAM, HYB1, HYB2 = 0, 1, 2, 3, 4
GUESS_PLAIN, GUESS_RK4, GUESS_EXTERNAL = 0, 1, 2
FIELDS_NONE, FIELDS_GRID, FIELDS_WALD = 0, 1, 2
DEPOSIT_CONSERVING, DEPOSIT_PAPER = 0, 1
SOLVER_PICARD, SOLVER_NEWTON = 0, 1
ALIVE, IMPLICIT, NOCONV, REMOVED, REFLECTED, NONFINITE = 1, 2, 4, 8, 16, 32
NPARAM = 5510


class PushParams(C.Structure):
    _fields_ = [("a", C.c_double), ("dt", C.c_double), ("pusher", C.c_int),
                ("guess", C.c_int), ("thr", C.c_double), ("tol", C.c_double),
                ("kmax", C.c_int), ("field_kind", C.c_int), ("B0", C.c_double),
                ("r_min", C.c_double), ("r_max", C.c_double),
                ("th_lo", C.c_double), ("th_hi", C.c_double),
                ("ham_eps", C.c_double), ("dt_impl", C.c_double), ("t_end", C.c_double),
                ("deposit_mode", C.c_int), ("solver", C.c_int)]


def push_params(a, dt, pusher=RK4, guess=GUESS_PLAIN, thr=0.0, tol=1e-13,
                kmax=50, field_kind=FIELDS_NONE, B0=0.0, r_min=0.0,
                r_max=1e300, th_lo=-1.0, th_hi=10.0, ham_eps=1e-10, dt_impl=0.0,
                t_end=0.0, deposit_mode=DEPOSIT_CONSERVING, solver=SOLVER_PICARD):
    return PushParams(a, dt, pusher, guess, thr, tol, kmax, field_kind, B0,
                      r_min, r_max, th_lo, th_hi, ham_eps, dt_impl, t_end, deposit_mode,
                      solver)


class _OmParticles(C.Structure):
    _fields_ = [("n", C.c_long)] + [(k, D_P) for k in
                                    ("r", "th", "ph", "ur", "uth", "uph", "qm",
                                     "w", "H0", "herr")] + \
               [("flags", I_P), ("iters", I_P), ("crit", D_P), ("t", D_P)]


class _OmFields(C.Structure):
    _fields_ = [(k, D_P * 3) for k in ("Dn", "Dh0", "Dh1", "Bm", "Bn", "Bh",
                                       "Jprev")] + [("rho", D_P)]


def lib():
    global _LIB
    if _LIB is None:
        path = os.path.join(_HERE, "liboracle.so")
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        L.om_grid_new.restype = C.c_void_p
        L.om_grid_new.argtypes = [C.c_double, C.c_int, C.c_int, C.c_double,
                                  C.c_double, C.c_double]
        L.om_grid_free.argtypes = [C.c_void_p]
        L.om_energy.restype = C.c_double
        L.om_uniform.restype = C.c_double
        L.om_uniform.argtypes = [C.c_uint64, C.c_uint64]
        L.om_mlp_loss_grad.restype = C.c_double
        L.om_step_imr.restype = C.c_int
        L.om_step_ham.restype = C.c_int
        L.om_inject.restype = C.c_long
        _LIB = L
    return _LIB


def _p(a):
    return a.ctypes.data_as(D_P)


def _ip(a):
    return a.ctypes.data_as(I_P)


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


def _ptrs(arrs):
    return (D_P * len(arrs))(*[_p(a) for a in arrs])


# ---------------------------------------------------------------- pointwise
def metric(a, r, th):
    out = np.zeros(13)
    lib().om_metric(C.c_double(a), C.c_double(r), C.c_double(th), _p(out))
    return out


def metric_deriv(a, r, th):
    out = np.zeros(12)
    lib().om_metric_deriv(C.c_double(a), C.c_double(r), C.c_double(th), _p(out))
    return out


def metric_divdiff(a, k, r0, t0, r1, t1):
    q = np.zeros(6)
    lib().om_metric_divdiff(C.c_double(a), k, C.c_double(r0), C.c_double(t0),
                            C.c_double(r1), C.c_double(t1), _p(q))
    return q


def energy(a, z):
    z = _f64(z)
    return lib().om_energy(C.c_double(a), _p(z))


def rhs(a, qm, z, D=(0, 0, 0), B=(0, 0, 0)):
    z, D, B = _f64(z), _f64(D), _f64(B)
    f = np.zeros(6)
    lib().om_rhs(C.c_double(a), C.c_double(qm), _p(z), _p(D), _p(B), _p(f))
    return f


def wald_fields(a, B0, r, th, a_field=None):
    """D^i, B^i of the Wald field; a_field (default a) is the spin of the
    potential of eq. Amu, a the spacetime's (Sec. 3.3 uses a_field = 0)."""
    D, B = np.zeros(3), np.zeros(3)
    af = a if a_field is None else a_field
    lib().om_wald_fields_spin(C.c_double(a), C.c_double(af), C.c_double(B0),
                              C.c_double(r), C.c_double(th), _p(D), _p(B))
    return D, B


def wald_potential(a, B0, r, th):
    A = np.zeros(4)
    lib().om_wald_potential(C.c_double(a), C.c_double(B0), C.c_double(r),
                            C.c_double(th), _p(A))
    return A


# --------------------------------------------------------------------- grid
class Grid:
    """Spherical Kerr-Schild Yee grid (r log-spaced, theta uniform)."""

    def __init__(self, a, nr, nth, r_in, r_out, th0=np.pi / 200):
        self.a, self.nr, self.nth = float(a), int(nr), int(nth)
        self.r_in, self.r_out, self.th0 = float(r_in), float(r_out), float(th0)
        self._h = lib().om_grid_new(self.a, self.nr, self.nth, self.r_in,
                                    self.r_out, self.th0)
        self.rn = np.zeros(nr + 1)
        self.rh = np.zeros(nr)
        self.tn = np.zeros(nth + 1)
        self.th = np.zeros(nth)
        lib().om_grid_coords(C.c_void_p(self._h), _p(self.rn), _p(self.rh),
                             _p(self.tn), _p(self.th))

    def __del__(self):
        if getattr(self, "_h", None) and _LIB is not None:
            _LIB.om_grid_free(C.c_void_p(self._h))
            self._h = None

    @property
    def h(self):
        return C.c_void_p(self._h)

    def shape(self, c):
        """(nT, nR) of component c: 0..5 = D^r,D^th,D^ph,B^r,B^th,B^ph; 6 = nodes."""
        nR, nT = C.c_int(), C.c_int()
        lib().om_comp_shape(self.h, c, C.byref(nR), C.byref(nT))
        return (nT.value, nR.value)

    def zeros(self, c):
        return np.zeros(self.shape(c))

    def densitize(self, c, arr, direction=+1):
        arr = _f64(arr)
        out = np.zeros_like(arr)
        lib().om_densitize(self.h, c, direction, _p(arr), _p(out))
        return out


def gather(grid, G, r, th):
    G = [_f64(g) for g in G]
    D, B = np.zeros(3), np.zeros(3)
    lib().om_gather(grid.h, _ptrs(G), C.c_double(r), C.c_double(th), _p(D),
                    _p(B))
    return D, B


# ---------------------------------------------------------------- particles
class Particles:
    """SoA particle state (float64 except flags/iters)."""

    KEYS = ("r", "th", "ph", "ur", "uth", "uph", "qm", "w", "H0", "herr", "crit")

    def __init__(self, n):
        self.n = int(n)
        for k in self.KEYS:
            setattr(self, k, np.zeros(self.n))
        self.crit[:] = np.nan
        self.flags = np.full(self.n, ALIVE, dtype=np.int32)
        self.iters = np.zeros(self.n, dtype=np.int32)
        self.t = None  # own clocks (an array) or none

    @classmethod
    def from_state(cls, z, qm, w=None, H0=None):
        z = np.atleast_2d(_f64(z))
        p = cls(z.shape[0])
        p.r[:], p.th[:], p.ph[:] = z[:, 0], z[:, 1], z[:, 2]
        p.ur[:], p.uth[:], p.uph[:] = z[:, 3], z[:, 4], z[:, 5]
        p.qm[:] = qm
        p.w[:] = 1.0 if w is None else w
        return p

    def state(self):
        return np.stack([self.r, self.th, self.ph, self.ur, self.uth, self.uph],
                        axis=1)

    def copy(self):
        q = Particles(self.n)
        for k in self.KEYS:
            getattr(q, k)[:] = getattr(self, k)
        q.flags[:] = self.flags
        q.iters[:] = self.iters
        q.t = None if self.t is None else self.t.copy()
        return q

    def _struct(self):
        for k in self.KEYS:
            assert getattr(self, k).dtype == np.float64 and getattr(self, k).flags.c_contiguous
        if self.t is not None:
            assert self.t.dtype == np.float64 and self.t.flags.c_contiguous
        s = _OmParticles(self.n, *[_p(getattr(self, k)) for k in self.KEYS[:10]],
                         _ip(self.flags), _ip(self.iters), _p(self.crit),
                         _p(self.t) if self.t is not None else None)
        return s


def push(P, particles, grid=None, G=None, guess=None, force=None):
    s = particles._struct()
    Gp = _ptrs([_f64(g) for g in G]) if G is not None else None
    gp = _p(_f64(guess)) if guess is not None else None
    fp = _ip(np.ascontiguousarray(force, dtype=np.int32)) if force is not None else None
    lib().om_push(C.byref(P), grid.h if grid is not None else None, Gp,
                  C.byref(s), gp, fp)


def step_rk4(P, qm, z, grid=None, G=None):
    z = _f64(z)
    out = np.zeros(6)
    W = C.c_double()
    Gp = _ptrs([_f64(g) for g in G]) if G is not None else None
    lib().om_step_rk4(C.byref(P), grid.h if grid else None, Gp, C.c_double(qm),
                      _p(z), _p(out), C.byref(W))
    return out, W.value


def step_imr(P, qm, z, guess=None, grid=None, G=None):
    z = _f64(z)
    out = np.zeros(6)
    W = C.c_double()
    Gp = _ptrs([_f64(g) for g in G]) if G is not None else None
    gs = _p(_f64(guess)) if guess is not None else None
    k = lib().om_step_imr(C.byref(P), grid.h if grid else None, Gp,
                          C.c_double(qm), _p(z), gs, _p(out), C.byref(W))
    return out, k, W.value


def step_ham(P, z, guess=None):
    z = _f64(z)
    out = np.zeros(6)
    gs = _p(_f64(guess)) if guess is not None else None
    k = lib().om_step_ham(C.byref(P), _p(z), gs, _p(out))
    return out, k


# ------------------------------------------------------------------ deposit
def dep_weights(grid, r, th, p, q, flat=False):
    W = np.zeros(4)
    lib().om_dep_weights(grid.h, C.c_double(r), C.c_double(th), p, q, int(flat),
                         _p(W))
    return W


def deposit(grid, dt, old, new, qw, mode=None):
    """old/new: (n,3) arrays of (r, theta, phi).  Returns densitized
    (rho, J^r, J^theta, J^phi) on their sub-grids."""
    old, new, qw = _f64(old), _f64(new), _f64(qw)
    n = old.shape[0]
    mode = np.ones(n, np.int32) if mode is None else np.ascontiguousarray(mode, np.int32)
    rho, Jr, Jt, Jp = grid.zeros(6), grid.zeros(0), grid.zeros(1), grid.zeros(6)
    cols = [np.ascontiguousarray(x[:, i]) for x in (old, new) for i in range(3)]
    lib().om_deposit(grid.h, C.c_double(dt), C.c_long(n), *[_p(c) for c in cols],
                     _p(qw), _ip(mode), _p(rho), _p(Jr), _p(Jt), _p(Jp))
    return rho, Jr, Jt, Jp


# ------------------------------------------------------------------ Maxwell
def _dshapes(grid):
    return [grid.shape(0), grid.shape(1), grid.shape(2)]


def _bshapes(grid):
    return [grid.shape(3), grid.shape(4), grid.shape(5)]


def compute_E(grid, D, B):
    E = [np.zeros(s) for s in _dshapes(grid)]
    lib().om_compute_E(grid.h, _ptrs([_f64(x) for x in D]),
                       _ptrs([_f64(x) for x in B]), _ptrs(E))
    return E


def compute_H(grid, B, D):
    H = [np.zeros(s) for s in _bshapes(grid)]
    lib().om_compute_H(grid.h, _ptrs([_f64(x) for x in B]),
                       _ptrs([_f64(x) for x in D]), _ptrs(H))
    return H


def _ab(absorber):
    return _p(_f64(absorber)) if absorber is not None else None


def faraday(grid, dt, Bin, E, absorber=None):
    Bout = [np.zeros(s) for s in _bshapes(grid)]
    lib().om_faraday(grid.h, C.c_double(dt), _ab(absorber),
                     _ptrs([_f64(x) for x in Bin]), _ptrs([_f64(x) for x in E]),
                     _ptrs(Bout))
    return Bout


def ampere(grid, dt, Din, H, Jd, absorber=None):
    Dout = [_f64(x).copy() for x in Din]
    lib().om_ampere(grid.h, C.c_double(dt), _ab(absorber),
                    _ptrs([_f64(x) for x in Din]), _ptrs([_f64(x) for x in H]),
                    _ptrs([_f64(x) for x in Jd]), _ptrs(Dout))
    return Dout


class Fields:
    """Field time levels of the two-chain leapfrog (non-densitized D^i, B^i;
    densitized J^{n+1/2} and rho^{n+1})."""

    LEVELS = ("Dn", "Dh0", "Dh1", "Bm", "Bn", "Bh")

    def __init__(self, grid):
        self.grid = grid
        for k in self.LEVELS:
            sh = _dshapes(grid) if k[0] == "D" else _bshapes(grid)
            setattr(self, k, [np.zeros(s) for s in sh])
        self.Jprev = [np.zeros(s) for s in _dshapes(grid)]
        self.rho = grid.zeros(6)

    @classmethod
    def uniform_levels(cls, grid, D, B):
        F = cls(grid)
        for k in ("Dn", "Dh0", "Dh1"):
            setattr(F, k, [_f64(x).copy() for x in D])
        for k in ("Bm", "Bn", "Bh"):
            setattr(F, k, [_f64(x).copy() for x in B])
        return F

    def copy(self):
        F = Fields(self.grid)
        for k in self.LEVELS + ("Jprev",):
            setattr(F, k, [x.copy() for x in getattr(self, k)])
        F.rho = self.rho.copy()
        return F

    def _struct(self):
        s = _OmFields()
        for k in self.LEVELS + ("Jprev",):
            arrs = getattr(self, k)
            for c in range(3):
                assert arrs[c].dtype == np.float64 and arrs[c].flags.c_contiguous
                getattr(s, k)[c] = _p(arrs[c])
        s.rho = _p(self.rho)
        return s


def pic_step(P, grid, F, particles=None, absorber=None, guess=None,
             force=None, push_mode=0):
    s = F._struct()
    ps = particles._struct() if particles is not None else None
    gp = _p(_f64(guess)) if guess is not None else None
    fp = _ip(np.ascontiguousarray(force, np.int32)) if force is not None else None
    if particles is None:
        push_mode = 1
    lib().om_pic_step(C.byref(P), grid.h, _ab(absorber), C.byref(s),
                      C.byref(ps) if ps is not None else None, gp, fp,
                      push_mode)


# -------------------------------------------------------------- diagnostics
def deposit_paper(grid, z, qw, mode=None):
    """The paper's current (Sec. 2.3) at the states z (n,6): densitized
    (rho, J^r, J^theta, J^phi) on their sub-grids."""
    z, qw = _f64(np.atleast_2d(z)), _f64(qw)
    n = z.shape[0]
    mode = np.ones(n, np.int32) if mode is None else np.ascontiguousarray(mode, np.int32)
    rho, Jr, Jt, Jp = grid.zeros(6), grid.zeros(0), grid.zeros(1), grid.zeros(6)
    cols = [np.ascontiguousarray(z[:, i]) for i in (0, 1, 3, 4, 5)]
    lib().om_deposit_paper(grid.h, C.c_long(n), *[_p(c) for c in cols], _p(qw), _ip(mode),
                           _p(rho), _p(Jr), _p(Jt), _p(Jp))
    return rho, Jr, Jt, Jp


def div_clean(grid, D, rho_d, iters):
    """Divergence cleaning (Sec. 2.4): returns the corrected copies of the
    plain D^i and phi at the nodes."""
    Dc = [_f64(x).copy() for x in D]
    phi = grid.zeros(6)
    lib().om_div_clean(grid.h, _ptrs(Dc), _p(_f64(rho_d)), C.c_int(iters), _p(phi))
    return Dc, phi


def gauss_residual(grid, D, rho_d):
    out = grid.zeros(6)
    lib().om_gauss_residual(grid.h, _ptrs([_f64(x) for x in D]),
                            _p(_f64(rho_d)), _p(out))
    return out


def div_B(grid, B):
    out = grid.zeros(5)
    lib().om_div_B(grid.h, _ptrs([_f64(x) for x in B]), _p(out))
    return out


def poynting(grid, D, B):
    out = np.zeros(grid.nr + 1)
    lib().om_poynting(grid.h, _ptrs([_f64(x) for x in D]),
                      _ptrs([_f64(x) for x in B]), _p(out))
    return out


# ------------------------------------------------------------- initial data
def wald_grid(grid, B0, a_field=None):
    D = [np.zeros(s) for s in _dshapes(grid)]
    B = [np.zeros(s) for s in _bshapes(grid)]
    af = grid.a if a_field is None else a_field
    lib().om_wald_grid(grid.h, C.c_double(B0), C.c_double(af), _ptrs(D), _ptrs(B))
    return D, B


class InjectParams(C.Structure):
    _fields_ = [("r0", C.c_double), ("r1", C.c_double), ("mult", C.c_double),
                ("density", C.c_double), ("theta", C.c_double), ("seed", C.c_uint64)]


def inject(grid, params, event, B, particles, room):
    """Pair injection (Sec. 3.3) into `particles` (appended, returns a new
    Particles) from the plain B^r, B^theta; at most `room` new particles."""
    p = particles
    out = np.zeros((max(room, 0), 8))
    flags = np.ascontiguousarray(p.flags, np.int32)
    made = lib().om_inject(grid.h, C.byref(params), C.c_uint64(event), _p(_f64(B[0])),
                           _p(_f64(B[1])), C.c_long(p.n), _p(p.r), _p(p.th), _p(p.qm),
                           _p(p.w), _ip(flags), C.c_long(room), _p(out))
    new = out[:made]
    q = Particles(p.n + made)
    for k in Particles.KEYS:
        getattr(q, k)[:p.n] = getattr(p, k)
    q.flags[:p.n], q.iters[:p.n] = p.flags, p.iters
    for i, k in enumerate(("r", "th", "ph", "ur", "uth", "uph", "qm", "w")):
        getattr(q, k)[p.n:] = new[:, i]
    q.H0[p.n:] = [energy(grid.a, z) for z in new[:, :6]]
    q.crit[p.n:] = np.nan
    return q


def split_monopole_grid(grid, B0, zeta0):
    D = [np.zeros(s) for s in _dshapes(grid)]
    B = [np.zeros(s) for s in _bshapes(grid)]
    lib().om_split_monopole_grid(grid.h, C.c_double(B0), C.c_double(zeta0),
                                 _ptrs(D), _ptrs(B))
    return D, B


def uniform(seed, counter):
    return lib().om_uniform(C.c_uint64(seed), C.c_uint64(counter))


INIT_ORBITS, INIT_SHELL_ISO, INIT_SHELL_MJ = 0, 1, 2


def init_particles(kind, a, seed, n, r0, r1, t0, t1, p0, w=1.0):
    p = Particles(n)
    s = p._struct()
    lib().om_init_particles(kind, C.c_double(a), C.c_uint64(seed), C.c_long(n),
                            C.c_double(r0), C.c_double(r1), C.c_double(t0),
                            C.c_double(t1), C.c_double(p0), C.c_double(w),
                            C.byref(s))
    return p


# ---------------------------------------------------------------------- MLP
def mlp_forward(theta, X):
    theta, X = _f64(theta), _f64(X)
    Y = np.zeros((X.shape[0], 6))
    lib().om_mlp_forward(_p(theta), C.c_long(X.shape[0]), _p(X), _p(Y))
    return Y


def mlp_loss_grad(theta, X, T):
    theta, X, T = _f64(theta), _f64(X), _f64(T)
    g = np.zeros(NPARAM)
    loss = lib().om_mlp_loss_grad(_p(theta), C.c_long(X.shape[0]), _p(X), _p(T),
                                  _p(g))
    return loss, g
