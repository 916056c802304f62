"""FP64 CPU oracle for the GRACE-DG collision operator -- TEST INFRASTRUCTURE.

Only the test suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  The product library never loads it and shares no code
with it.

The nested quadrature itself is plain C (``oracle.c``, built into
``liboracle.so`` by :func:`build`); this module wraps it with ctypes and adds the
pieces that are most readable in numpy:

* the Gauss-Legendre rule, taken from ``numpy.polynomial.legendre.leggauss``
  (a library routine), Sec. 3.3 Eq. quad;
* the projection of an initial profile onto the Legendre basis, Sec. 3.2
  Eq. init, with 16 points per bin;
* the moments M_p and the error norms e_c, e_d of Sec. 4.1;
* closed-form solutions used as pins: the constant kernel (Sec. 4.2,
  Eq. fcoagsolution), the additive kernel from f0 = e^-x (the textbook Golovin
  form; the paper's additive test uses a monodisperse start instead), and the
  multiplicative-kernel pure fragmentation (Sec. 4.4, Eq. fragsolution).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

# enum values of oracle.c
KERNELS = {"const": 0, "additive": 1, "multiplicative": 2, "ballistic": 3, "maxwell": 4}
FRAGS = {"none": 0, "powerlaw": 1, "uniform_binary": 2, "remnant_only": 3, "general": 4}


def build(force: bool = True) -> str:
    """Compile the C oracle (plain gcc, -O2, OpenMP across cells)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", _SRC,
                               "-o", _LIB + ".tmp", "-lm"])
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cfg(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int), ("k", ctypes.c_int), ("Q", ctypes.c_int),
                ("s", ctypes.POINTER(ctypes.c_double)), ("w", ctypes.POINTER(ctypes.c_double)),
                ("xmin", ctypes.c_double), ("xmax", ctypes.c_double),
                ("conservative", ctypes.c_int), ("kern", ctypes.c_int), ("v0", ctypes.c_double),
                ("frag", ctypes.c_int), ("alpha", ctypes.c_double), ("vb", ctypes.c_double)]


_lib = None


NATIVE_FLAGS = ["-O3", "-march=native", "-fopenmp"]


def use_native() -> str:
    """Compile the same source with -O3 -march=native for the host this runs on and use
    that build from now on (the CPU-baseline timing; the tests keep the portable -O2
    build).  Returns the compiler flags."""
    global _lib
    import tempfile
    path = os.path.join(tempfile.gettempdir(), f"liboracle_native_{os.getpid()}.so")
    subprocess.check_call(["gcc", *NATIVE_FLAGS, "-fPIC", "-shared", _SRC, "-o", path, "-lm"])
    _lib = None
    _load(path)
    return " ".join(NATIVE_FLAGS)


def _load(path=None):
    global _lib
    if _lib is None:
        if path is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build(force=True)
            path = _LIB
        lib = ctypes.CDLL(path)
        dp = ctypes.POINTER(ctypes.c_double)
        cp = ctypes.POINTER(_Cfg)
        lib.oracle_set_threads.argtypes = [ctypes.c_int]
        lib.oracle_set_threads.restype = ctypes.c_int
        lib.oracle_n_out.argtypes = [cp]
        lib.oracle_n_out.restype = ctypes.c_int
        lib.oracle_rates.argtypes = [cp, ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     dp, dp, dp]
        lib.oracle_rates.restype = ctypes.c_int
        lib.oracle_edges.argtypes = [cp, dp]
        lib.oracle_edges.restype = ctypes.c_int
        lib.oracle_flux_points.argtypes = [cp, dp, ctypes.c_double, ctypes.c_double, ctypes.c_int, dp, dp]
        lib.oracle_flux_points.restype = ctypes.c_int
        lib.oracle_rhs.argtypes = [cp, ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_int, dp, dp, dp, dp]
        lib.oracle_rhs.restype = ctypes.c_int
        lib.oracle_limit.argtypes = [cp, ctypes.c_int, dp]
        lib.oracle_limit.restype = ctypes.c_long
        lib.oracle_rk.argtypes = [cp, ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_int, dp,
                                  ctypes.c_double, ctypes.c_int]
        lib.oracle_rk.restype = ctypes.c_long
        lib.oracle_rk_trace.argtypes = [cp, ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_int, dp,
                                        ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_ulonglong)]
        lib.oracle_rk_trace.restype = ctypes.c_long
        lib.oracle_rk_adaptive.argtypes = [cp, ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_int, dp,
                                           ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                           ctypes.c_int, dp]
        lib.oracle_rk_adaptive.restype = ctypes.c_long
        lib.oracle_cfl_dt.argtypes = [cp, ctypes.c_int, dp, dp, dp, ctypes.c_double, ctypes.c_int, dp]
        lib.oracle_cfl_dt.restype = ctypes.c_double
        lib.oracle_inner.argtypes = [cp, ctypes.c_double, ctypes.c_double, ctypes.c_double, dp, dp]
        lib.oracle_inner.restype = ctypes.c_int
        _lib = lib
    return _lib


def _dp(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@dataclass
class Config:
    """One DG discretisation of the collision operator (Secs. 3.1-3.3)."""
    N: int
    k: int
    xmin: float
    xmax: float
    kernel: str = "const"
    frag: str = "none"
    conservative: bool = False
    Q: int = 0                  # 0 -> k+1 (Sec. 3.3)
    v0: float = 1.0
    alpha: float = -11.0 / 6.0
    vfrag: float = 0.5          # threshold when no per-cell value is given
    vb: float = 0.0             # bouncing threshold (Maxwellian kernel, Sec. 4.5)
    levels: tuple = ()          # per-cell threshold table (>= 2 entries) or empty
    _keep: list = field(default_factory=list, repr=False)

    @property
    def q(self) -> int:
        return self.Q if self.Q > 0 else self.k + 1

    @property
    def P(self) -> int:
        return self.N * (self.k + 1)

    def _c(self):
        s, w = np.polynomial.legendre.leggauss(self.q)
        s = np.ascontiguousarray(s, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        self._keep = [s, w]
        c = _Cfg(self.N, self.k, self.q, _dp(s), _dp(w), float(self.xmin), float(self.xmax),
                 int(bool(self.conservative)), KERNELS[self.kernel], float(self.v0),
                 FRAGS[self.frag], float(self.alpha), float(self.vb))
        return c

    @property
    def n_out(self) -> int:
        return _load().oracle_n_out(ctypes.byref(self._c()))

    def _levels(self):
        if len(self.levels) >= 2:
            lv = np.ascontiguousarray(self.levels, dtype=np.float64)
            return len(lv), lv
        return 0, None


def set_threads(n: int) -> int:
    """OpenMP threads of the batch loops (n <= 0 keeps the current setting); returns
    the number in use."""
    return int(_load().oracle_set_threads(int(n)))


def edges(cfg: Config) -> np.ndarray:
    e = np.zeros(cfg.N + 1)
    c = cfg._c()
    assert _load().oracle_edges(ctypes.byref(c), _dp(e)) == 0
    return e


def _cells(cfg, g, kscale, vfrag):
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(-1, cfg.P))
    C = g.shape[0]
    ks = None if kscale is None else np.ascontiguousarray(np.broadcast_to(np.asarray(kscale, np.float64), (C,)))
    vf = None if vfrag is None else np.ascontiguousarray(np.broadcast_to(np.asarray(vfrag, np.float64), (C,)))
    return g, C, ks, vf


def rhs(cfg: Config, g, kscale=None, vfrag=None):
    """Raw flux vector Y [C, n_out], right-hand side L [C, P], edge fluxes [C, N+1].

    Y = (F(e_1)..F(e_{N-1}), F(e_N) if non-conservative, V_{j,i} for j<N, 1<=i<=k)."""
    g, C, ks, vf = _cells(cfg, g, kscale, vfrag)
    no = cfg.n_out
    Y = np.zeros((C, no))
    L = np.zeros((C, cfg.P))
    Fe = np.zeros((C, cfg.N + 1))
    nl, lv = cfg._levels()
    c = cfg._c()
    rc = _load().oracle_rhs(ctypes.byref(c), C, _dp(g), _dp(ks), _dp(vf), float(cfg.vfrag), nl, _dp(lv),
                            _dp(Y), _dp(L), _dp(Fe))
    assert rc == 0
    return Y, L, Fe


def flux_points(cfg: Config, g, xs, kscale=1.0, vfrag=None):
    g = np.ascontiguousarray(np.asarray(g, dtype=np.float64).reshape(cfg.P))
    xs = np.ascontiguousarray(np.asarray(xs, dtype=np.float64))
    F = np.zeros_like(xs)
    c = cfg._c()
    rc = _load().oracle_flux_points(ctypes.byref(c), _dp(g), float(kscale),
                                    float(cfg.vfrag if vfrag is None else vfrag), len(xs), _dp(xs), _dp(F))
    assert rc == 0
    return F


def limit(cfg: Config, g):
    """Scaling limiter (Eqs. recon, gamma) on a copy; returns (limited, violations)."""
    g = np.array(np.asarray(g, dtype=np.float64).reshape(-1, cfg.P), copy=True)
    c = cfg._c()
    v = _load().oracle_limit(ctypes.byref(c), g.shape[0], _dp(g))
    assert v >= 0
    return g, int(v)


def rk(cfg: Config, g, dt: float, n_steps: int, kscale=None, vfrag=None):
    """n_steps of SSP-RK3 (Eq. RK3), limiter on the start state and after every stage."""
    g, C, ks, vf = _cells(cfg, g, kscale, vfrag)
    g = g.copy()
    nl, lv = cfg._levels()
    c = cfg._c()
    v = _load().oracle_rk(ctypes.byref(c), C, _dp(g), _dp(ks), _dp(vf), float(cfg.vfrag), nl, _dp(lv),
                          float(dt), int(n_steps))
    assert v >= 0
    return g, int(v)


def advect(cfg: Config, g, vel, dt: float, dx: float, periodic: bool = True):
    """Transport between the hydro cells of a row, the hydro half of operator splitting
    (Sec. 5.2): every Legendre coefficient of bin j moves with the bin's velocity vel[j]
    by first-order upwind finite volumes, Courant number c = vel[j] dt / dx (|c| <= 1):
    g_c <- (1 - |c|) g_c + |c| g_up, up = c - 1 for vel >= 0 and c + 1 otherwise;
    periodic wraps the row, otherwise nothing flows in at its ends."""
    g = np.asarray(g, dtype=np.float64).reshape(-1, cfg.N, cfg.k + 1)
    C = g.shape[0]
    out = np.empty_like(g)
    for c in range(C):
        for j in range(cfg.N):
            cj = vel[j] * dt / dx
            a = abs(cj)
            assert a <= 1.0
            up = c - 1 if cj >= 0.0 else c + 1
            if 0 <= up < C:
                gu = g[up, j]
            elif periodic:
                gu = g[up % C, j]
            else:
                gu = np.zeros(cfg.k + 1)
            out[c, j] = (1.0 - a) * g[c, j] + a * gu
    return out.reshape(C, -1)


def split_step(cfg: Config, g, vel, dx: float, dt: float, n_steps: int, kscale=None, vfrag=None,
               periodic: bool = True):
    """Strang splitting of transport and collisions: per step, transport over dt/2, one
    SSP-RK3 step over dt (rk(): start limiter, limiter after every stage), transport over
    dt/2.  Returns (g, violations)."""
    g = np.asarray(g, dtype=np.float64).reshape(-1, cfg.P)
    viol = 0
    for _ in range(n_steps):
        g = advect(cfg, g, vel, 0.5 * dt, dx, periodic)
        g, v = rk(cfg, g, dt, 1, kscale=kscale, vfrag=vfrag)
        viol += v
        g = advect(cfg, g, vel, 0.5 * dt, dx, periodic)
    return g, viol


def rk_traced(cfg: Config, g, dt: float, n_steps: int, kscale=None, vfrag=None):
    """rk() that also returns, per cell, a hash of every (limiter call, bin) where the
    limiter changed the state: equal hashes mean the same active set."""
    g, C, ks, vf = _cells(cfg, g, kscale, vfrag)
    g = g.copy()
    tr = np.zeros(C, dtype=np.uint64)
    nl, lv = cfg._levels()
    c = cfg._c()
    v = _load().oracle_rk_trace(ctypes.byref(c), C, _dp(g), _dp(ks), _dp(vf), float(cfg.vfrag), nl, _dp(lv),
                                float(dt), int(n_steps), tr.ctypes.data_as(ctypes.POINTER(ctypes.c_ulonglong)))
    assert v >= 0
    return g, int(v), tr


def rk_adaptive(cfg: Config, g, cfl: float, dt_max: float, t_end: float, n_sub: int, t=None,
                kscale=None, vfrag=None, floor: float = 0.0):
    """n_sub sub-steps of SSP-RK3 with a per-cell step under the CFL bound (Eq. dt):
    dt_c = min(dt_max, t_end - t_c, cfl * B_c), B_c the bound over the bins losing
    mass at the sub-step's start (more than floor times the cell's largest edge
    flux).  Returns (g, t, violations); t (per cell, default zeros) is the time each
    cell has reached."""
    g, C, ks, vf = _cells(cfg, g, kscale, vfrag)
    g = g.copy()
    t = np.zeros(C) if t is None else np.ascontiguousarray(t, dtype=np.float64).copy()
    assert t.shape == (C,)
    nl, lv = cfg._levels()
    c = cfg._c()
    v = _load().oracle_rk_adaptive(ctypes.byref(c), C, _dp(g), _dp(ks), _dp(vf), float(cfg.vfrag), nl, _dp(lv),
                                   float(cfl), float(dt_max), float(floor), float(t_end), int(n_sub), _dp(t))
    assert v >= 0
    return g, t, int(v)


def inner(cfg: Config, x: float, u: float, v: float):
    """(int_x^{u+v} w b dw, int_{x_min}^x w b dw) at one point (App. B)."""
    pw = np.zeros(1)
    nw = np.zeros(1)
    c = cfg._c()
    _load().oracle_inner(ctypes.byref(c), float(x), float(u), float(v), _dp(pw), _dp(nw))
    return float(pw[0]), float(nw[0])


def rates(cfg: Config, u: float, v: float, kscale: float = 1.0, vfrag=None):
    """(K_coag, K_frag, m_frag of the general law) at one node pair (Sec. 4.5, Eq. mfrag)."""
    out = [np.zeros(1) for _ in range(3)]
    c = cfg._c()
    vf = cfg.vfrag if vfrag is None else vfrag
    _load().oracle_rates(ctypes.byref(c), float(u), float(v), float(kscale), float(vf), *(_dp(o) for o in out))
    return tuple(float(o[0]) for o in out)


def cfl_dt(cfg: Config, g, kscale=None, vfrag=None) -> float:
    g, C, ks, vf = _cells(cfg, g, kscale, vfrag)
    nl, lv = cfg._levels()
    c = cfg._c()
    return float(_load().oracle_cfl_dt(ctypes.byref(c), C, _dp(g), _dp(ks), _dp(vf), float(cfg.vfrag), nl, _dp(lv)))


# ----------------------------------------------------------------- Eq. init
def project(cfg: Config, g0, R: int = 16) -> np.ndarray:
    """g_j^i = (2i+1)/2 * sum_a w_a g0(c_j + h_j s_a / 2) P_i(s_a), R points per bin."""
    e = edges(cfg)
    s, w = np.polynomial.legendre.leggauss(R)
    h = np.diff(e)
    c = 0.5 * (e[:-1] + e[1:])
    x = c[:, None] + 0.5 * h[:, None] * s[None, :]
    vals = g0(x)
    out = np.zeros((cfg.N, cfg.k + 1))
    for i in range(cfg.k + 1):
        Pi = np.polynomial.legendre.Legendre.basis(i)(s)
        out[:, i] = (2 * i + 1) / 2.0 * (vals * (w * Pi)[None, :]).sum(axis=1)
    return out.reshape(cfg.P)


def evaluate(cfg: Config, g, x) -> np.ndarray:
    """DG polynomial at masses x (each x is evaluated in the bin that contains it)."""
    e = edges(cfg)
    g = np.asarray(g).reshape(cfg.N, cfg.k + 1)
    x = np.asarray(x, dtype=np.float64)
    j = np.clip(np.searchsorted(e, x, side="right") - 1, 0, cfg.N - 1)
    h = e[j + 1] - e[j]
    xi = 2.0 * (x - 0.5 * (e[j] + e[j + 1])) / h
    out = np.zeros_like(x)
    for i in range(cfg.k + 1):
        out += g[j, i] * np.polynomial.legendre.Legendre.basis(i)(xi)
    return out


# ------------------------------------------------------------ Sec. 4.1 diagnostics
def moments(cfg: Config, g, p: int, R: int = 32) -> np.ndarray:
    """M_p = sum_j sum_i g_j^i int_{I_j} x^(p-1) P_i(xi) dx  (per cell)."""
    e = edges(cfg)
    s, w = np.polynomial.legendre.leggauss(R)
    h = np.diff(e)
    c = 0.5 * (e[:-1] + e[1:])
    x = c[:, None] + 0.5 * h[:, None] * s[None, :]
    W = np.zeros((cfg.N, cfg.k + 1))
    for i in range(cfg.k + 1):
        Pi = np.polynomial.legendre.Legendre.basis(i)(s)
        W[:, i] = 0.5 * h * ((x ** (p - 1)) * (w * Pi)[None, :]).sum(axis=1)
    g = np.asarray(g).reshape(-1, cfg.N, cfg.k + 1)
    return (g * W[None]).sum(axis=(1, 2))


def error_c(cfg: Config, g, exact, R: int = 16) -> float:
    """e_c = sum_j h_j/2 sum_a w_a |g_j(x_j^a) - g(x_j^a)|."""
    e = edges(cfg)
    s, w = np.polynomial.legendre.leggauss(R)
    h = np.diff(e)
    c = 0.5 * (e[:-1] + e[1:])
    x = c[:, None] + 0.5 * h[:, None] * s[None, :]
    gn = np.asarray(g).reshape(cfg.N, cfg.k + 1)
    num = np.zeros_like(x)
    for i in range(cfg.k + 1):
        num += gn[:, i:i + 1] * np.polynomial.legendre.Legendre.basis(i)(s)[None, :]
    return float((0.5 * h[:, None] * w[None, :] * np.abs(num - exact(x))).sum())


def error_d(cfg: Config, g, exact) -> float:
    """e_d = sum_j h_j |g_j(xhat_j) - g(xhat_j)|, xhat_j the geometric mean of the bin."""
    e = edges(cfg)
    xh = np.sqrt(e[:-1] * e[1:])
    return float((np.diff(e) * np.abs(evaluate(cfg, g, xh) - exact(xh))).sum())


# ------------------------------------------------------------ closed forms (pins)
def g_const(x, tau):
    """Constant kernel, f(x,0) = e^-x: f = 4/(2+tau)^2 exp(-2x/(2+tau)); g = x f (Sec. 4.2)."""
    return x * 4.0 / (2.0 + tau) ** 2 * np.exp(-2.0 * x / (2.0 + tau))


def g_additive(x, tau):
    """Additive kernel K = x+y, f(x,0) = e^-x (Golovin):
    f = (1-T)/(x sqrt T) exp(-(1+T) x) I_1(2 x sqrt T), T = 1 - e^-tau;  g = x f."""
    from scipy.special import i1e
    T = 1.0 - np.exp(-tau)
    z = 2.0 * x * np.sqrt(T)
    # I_1(z) e^{-(1+T)x} = i1e(z) e^{z - (1+T) x}
    return (1.0 - T) / np.sqrt(T) * i1e(z) * np.exp(z - (1.0 + T) * x)


def g_ziff(x, tau):
    """K_frag = xy with uniform binary breakage, f(x,0) = e^-x:
    f = (1+tau)^2 exp(-x (1+tau)); g = x f (Sec. 4.4, Eq. fragsolution)."""
    return x * (1.0 + tau) ** 2 * np.exp(-x * (1.0 + tau))
