"""Python binding of ``libgracedg.so`` (ctypes, argument marshalling only).

Every numerical step runs in the HIP library; this module turns torch tensors
into device pointers and Python values into the C structs of ``gracedg.h``.
There is no fallback: if the library is missing the import of any call raises.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# GRACEDG_LIBRARY=checks selects the build with the device checks (gd_plan_checks)
LIB_PATH = os.path.join(_HERE, "libgracedg_checks.so" if os.environ.get("GRACEDG_LIBRARY") == "checks"
                        else "libgracedg.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "gracedg.h")

GD_OK, GD_EINVAL, GD_EHIP, GD_ENOMEM, GD_EUNSUPPORTED, GD_EPOSITIVITY = 0, -1, -2, -3, -4, -5
KERNELS = {"const": 0, "additive": 1, "multiplicative": 2, "ballistic": 3, "maxwell": 4}
FRAGS = {"none": 0, "powerlaw": 1, "uniform_binary": 2, "remnant_only": 3, "general": 4}
PREC = {"fp64": 0, "mixed": 1}


class GDError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gracedg error {code}: {msg}")
        self.code = code


class _Kernel(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("v0", ctypes.c_double), ("v_bounce", ctypes.c_double)]


class _Frag(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("alpha", ctypes.c_double), ("n_levels", ctypes.c_int),
                ("levels", ctypes.POINTER(ctypes.c_double))]


class _Grid(ctypes.Structure):
    _fields_ = [("x_min", ctypes.c_double), ("x_max", ctypes.c_double), ("conservative", ctypes.c_int),
                ("quad_points", ctypes.c_int)]


class _Info(ctypes.Structure):
    _fields_ = [("bins", ctypes.c_int), ("order", ctypes.c_int), ("P", ctypes.c_int), ("n_out", ctypes.c_int),
                ("n_levels", ctypes.c_int), ("nnz_folded", ctypes.c_longlong),
                ("flops_per_eval", ctypes.c_double), ("device_bytes", ctypes.c_size_t)]


_lib = None
_VP = ctypes.c_void_p
_DP = ctypes.POINTER(ctypes.c_double)


def declared_symbols():
    """Names of every function declared in include/gracedg.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(gd_[a-z_0-9]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2607_13740_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "gd_init_tensor": ([ctypes.POINTER(_Kernel), ctypes.POINTER(_Frag), ctypes.c_int, ctypes.c_int,
                                ctypes.POINTER(_Grid), ctypes.POINTER(_VP)], ctypes.c_int),
            "gd_tensor_info": ([_VP, ctypes.POINTER(_Info)], ctypes.c_int),
            "gd_tensor_export": ([_VP, ctypes.c_int, _DP], ctypes.c_int),
            "gd_tensor_edges": ([_VP, _DP], ctypes.c_int),
            "gd_free_tensor": ([_VP], None),
            "gd_plan_create": ([ctypes.POINTER(_VP), ctypes.POINTER(ctypes.c_int), ctypes.c_int, ctypes.c_int,
                                _DP, _VP, ctypes.POINTER(_VP)], ctypes.c_int),
            "gd_plan_schedule_stats": ([_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                                        ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
            "gd_plan_sizes": ([_VP, ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_longlong)],
                              ctypes.c_int),
            "gd_plan_destroy": ([_VP], None),
            "gd_collision_rhs": ([_VP, _VP, _VP, _VP, _VP], ctypes.c_int),
            "gd_tensor_upload": ([_VP], ctypes.c_int),
            "gd_plan_set_vfrag": ([_VP, _DP], ctypes.c_int),
            "gd_advect": ([_VP, _VP, _DP, ctypes.c_double, ctypes.c_double, ctypes.c_int], ctypes.c_int),
            "gd_split_step": ([_VP, _VP, _VP, _DP, ctypes.c_double, ctypes.c_int, ctypes.c_double, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
            "gd_plan_set_lanes": ([_VP, ctypes.c_int], ctypes.c_int),
            "gd_plan_checks": ([_VP, ctypes.POINTER(ctypes.c_uint)], ctypes.c_int),
            "gd_plan_group_rows": ([_VP, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
            "gd_plan_lanes": ([_VP, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
            "gd_collision_rhs_noalloc": ([_VP, ctypes.c_int, ctypes.c_int, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
            "gd_rk_step": ([_VP, _VP, _VP, ctypes.c_double, ctypes.c_int,
                            ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
            "gd_rk_advance": ([_VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                               ctypes.c_double, ctypes.c_int, ctypes.POINTER(ctypes.c_longlong),
                               ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
            "gd_projection_points": ([_VP, _DP], ctypes.c_int),
            "gd_project": ([_VP, ctypes.c_int, _VP, _VP, _VP], ctypes.c_int),
            "gd_plan_timing": ([_VP, ctypes.c_int], ctypes.c_int),
            "gd_plan_set_variant": ([_VP, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int], ctypes.c_int),
            "gd_plan_variant": ([_VP] + [ctypes.POINTER(ctypes.c_int)] * 5 + [_DP], ctypes.c_int),
            "gd_plan_autotune": ([_VP, _VP, _VP, ctypes.c_char_p] + [ctypes.POINTER(ctypes.c_int)] * 4, ctypes.c_int),
            "gd_plan_use_graph": ([_VP, ctypes.c_int], ctypes.c_int),
            "gd_plan_bins": ([_VP, ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
            "gd_plan_algorithmic_flops": ([_VP, _DP], ctypes.c_int),
            "gd_rk_forward": ([_VP, _VP, _VP, ctypes.c_double, ctypes.c_int, _VP, _VP,
                               ctypes.POINTER(ctypes.c_longlong)], ctypes.c_int),
            "gd_adjoint": ([_VP, _VP, _VP, _VP, ctypes.c_double, ctypes.c_int, _VP, _VP, _VP], ctypes.c_int),
            "gd_collision_vjp": ([_VP, _VP, _VP, _VP, _VP, _VP, _VP], ctypes.c_int),
            "gd_plan_contraction_time": ([_VP, _DP, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
            "gd_plan_stage_time": ([_VP, _DP, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
            "gd_last_error": ([], ctypes.c_char_p),
        }
        for name, (args, res) in sig.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _check(rc, counted=False):
    """Raise on a failed call.  counted: the call was given a violation counter, so
    GD_EPOSITIVITY (completed, with limiter violations counted) is a result, not an error."""
    if rc != GD_OK and not (counted and rc == GD_EPOSITIVITY):
        raise GDError(rc, lib().gd_last_error().decode())


def _ptr(t):
    """Device (or host) address of a torch tensor, or NULL."""
    if t is None:
        return None
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _dev64(t, n, name):
    import torch
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
        raise TypeError(f"{name} must be a float64 device tensor")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    return _ptr(t)


class Tensor:
    """Collision tensor for one kernel, fragment law, grid and order (gd_init_tensor)."""

    def __init__(self, bins, order, x_min, x_max, kernel="const", frag="none", alpha=-11.0 / 6.0,
                 levels=(0.5,), v0=1.0, conservative=False, quad_points=0, v_bounce=0.0):
        self.levels = np.ascontiguousarray(levels, dtype=np.float64)
        k = _Kernel(KERNELS[kernel], float(v0), float(v_bounce))
        f = _Frag(FRAGS[frag], float(alpha), int(len(self.levels)),
                  self.levels.ctypes.data_as(_DP))
        g = _Grid(float(x_min), float(x_max), int(bool(conservative)), int(quad_points))
        h = _VP()
        _check(lib().gd_init_tensor(ctypes.byref(k), ctypes.byref(f), int(bins), int(order), ctypes.byref(g),
                                    ctypes.byref(h)))
        self.h = h
        self.bins, self.order = int(bins), int(order)
        self.conservative = bool(conservative)
        inf = self.info()
        self.P, self.n_out, self.n_levels = inf["P"], inf["n_out"], inf["n_levels"]

    def info(self):
        i = _Info()
        _check(lib().gd_tensor_info(self.h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _Info._fields_}

    def export(self, level=0):
        out = np.zeros((self.n_out, self.P, self.P))
        _check(lib().gd_tensor_export(self.h, int(level), out.ctypes.data_as(_DP)))
        return out

    def edges(self):
        out = np.zeros(self.bins + 1)
        _check(lib().gd_tensor_edges(self.h, out.ctypes.data_as(_DP)))
        return out

    def projection_points(self):
        out = np.zeros((self.bins, 16))
        _check(lib().gd_projection_points(self.h, out.ctypes.data_as(_DP)))
        return out

    def project(self, samples, out=None, stream=None):
        """samples: float64 device tensor [C, bins, 16] of g0 at projection_points()."""
        import torch
        C = samples.shape[0]
        if out is None:
            out = torch.empty((C, self.P), dtype=torch.float64, device=samples.device)
        _dev64(samples, C * self.bins * 16, "samples")
        _dev64(out, C * self.P, "out")
        st = stream if stream is not None else torch.cuda.current_stream(samples.device).cuda_stream
        _check(lib().gd_project(self.h, int(C), _ptr(samples), _ptr(out), ctypes.c_void_p(st)))
        return out

    def upload(self):
        """Device layouts of both contraction precisions now (gd_tensor_upload)."""
        _check(lib().gd_tensor_upload(self.h))
        return self

    def collision_rhs_noalloc(self, g, precision="mixed", kscale=None, rhs=None, raw=None, stream=None):
        """L[g] of the cells in g ([C*P] float64 device) with level 0 of the threshold
        table and no allocation in the library (gd_collision_rhs_noalloc); rhs (and raw,
        [C*n_out]) are the caller's."""
        import torch
        C = g.numel() // self.P
        if C * self.P != g.numel():
            raise ValueError("g must hold whole cells")
        if rhs is None:
            rhs = torch.empty_like(g)
        _dev64(g, C * self.P, "g")
        _dev64(rhs, C * self.P, "rhs")
        _dev64(kscale, C, "kscale")
        _dev64(raw, C * self.n_out, "raw")
        st = stream if stream is not None else torch.cuda.current_stream(g.device).cuda_stream
        _check(lib().gd_collision_rhs_noalloc(self.h, PREC[precision], int(C), _ptr(g), _ptr(kscale), _ptr(rhs),
                                              _ptr(raw), ctypes.c_void_p(st)))
        return rhs

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.gd_free_tensor(h)
            self.h = None


class Plan:
    """Groups of hydro cells bound to tensors, one precision, one stream (gd_plan_create).

    vfrag: optional per-cell fragmentation thresholds (host array, all cells in plan
    order), used by tensors with several threshold levels."""

    def __init__(self, tensors, cells, precision="fp64", vfrag=None, stream=None):
        import torch
        if isinstance(tensors, Tensor):
            tensors, cells = [tensors], [cells]
        self.tensors = list(tensors)
        self.cells = [int(c) for c in cells]
        self.precision = precision
        arr_t = (_VP * len(self.tensors))(*[t.h for t in self.tensors])
        arr_c = (ctypes.c_int * len(self.cells))(*self.cells)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        vf = None
        self._vfrag = None
        if vfrag is not None:
            self._vfrag = np.ascontiguousarray(vfrag, dtype=np.float64)
            if self._vfrag.size != sum(self.cells):
                raise ValueError("vfrag needs one value per cell")
            vf = self._vfrag.ctypes.data_as(_DP)
        h = _VP()
        _check(lib().gd_plan_create(arr_t, arr_c, len(self.tensors), PREC[precision], vf, ctypes.c_void_p(stream),
                                    ctypes.byref(h)))
        self.h = h
        nc, nv = ctypes.c_longlong(), ctypes.c_longlong()
        _check(lib().gd_plan_sizes(self.h, ctypes.byref(nc), ctypes.byref(nv)))
        self.n_cells, self.n_values = nc.value, nv.value
        self.n_raw = sum(c * t.n_out for t, c in zip(self.tensors, self.cells))
        nb = ctypes.c_longlong()
        _check(lib().gd_plan_bins(self.h, ctypes.byref(nb)))
        self.n_bins = nb.value

    def set_vfrag(self, vfrag):
        """New per-cell fragmentation thresholds (host values, all cells in plan order;
        None = the first level): brackets and blend weights rebuilt (gd_plan_set_vfrag)."""
        if vfrag is None:
            _check(lib().gd_plan_set_vfrag(self.h, None))
            self._vfrag = None
            return
        v = np.ascontiguousarray(vfrag, dtype=np.float64).reshape(-1)
        if v.size != self.n_cells:
            raise ValueError("vfrag needs one value per cell")
        _check(lib().gd_plan_set_vfrag(self.h, v.ctypes.data_as(_DP)))
        self._vfrag = v

    @property
    def vfrag(self):
        """The thresholds the plan's brackets were built from (None: the first level)."""
        return self._vfrag

    def schedule_stats(self, group=0):
        fm, ff, ns = ctypes.c_longlong(), ctypes.c_longlong(), ctypes.c_int()
        _check(lib().gd_plan_schedule_stats(self.h, int(group), ctypes.byref(fm), ctypes.byref(ff), ctypes.byref(ns)))
        return {"frags_mixed": fm.value, "frags_fp64": ff.value, "n_slots": ns.value}

    def collision_rhs(self, g, kscale=None, rhs=None, raw=None):
        import torch
        if rhs is None:
            rhs = torch.empty_like(g)
        _dev64(g, self.n_values, "g")
        _dev64(rhs, self.n_values, "rhs")
        _dev64(kscale, self.n_cells, "kscale")
        _dev64(raw, self.n_raw, "raw")
        _check(lib().gd_collision_rhs(self.h, _ptr(g), _ptr(kscale), _ptr(rhs), _ptr(raw)))
        return rhs

    def rk_step(self, g, dt, n_steps=1, kscale=None, count_violations=False):
        _dev64(g, self.n_values, "g")
        _dev64(kscale, self.n_cells, "kscale")
        v = ctypes.c_longlong(0)
        _check(lib().gd_rk_step(self.h, _ptr(g), _ptr(kscale), float(dt), int(n_steps),
                                ctypes.byref(v) if count_violations else None), counted=count_violations)
        return v.value if count_violations else None

    def _vel(self, vel):
        v = np.ascontiguousarray(vel, dtype=np.float64).reshape(-1)
        nb = sum(t.bins for t in self.tensors)
        if v.size != nb:
            raise ValueError(f"vel needs one velocity per bin of every group ({nb})")
        return v

    def advect(self, g, vel, dt, dx, periodic=True):
        """Upwind transport of every coefficient between neighbouring cells (gd_advect)."""
        _dev64(g, self.n_values, "g")
        v = self._vel(vel)
        _check(lib().gd_advect(self.h, _ptr(g), v.ctypes.data_as(_DP), float(dt), float(dx), int(bool(periodic))))

    def split_step(self, g, vel, dx, dt, n_steps=1, kscale=None, periodic=True, count_violations=False):
        """Strang splitting: transport dt/2, SSP-RK3 collision step dt, transport dt/2 (gd_split_step)."""
        _dev64(g, self.n_values, "g")
        _dev64(kscale, self.n_cells, "kscale")
        v = self._vel(vel)
        cnt = ctypes.c_longlong(0)
        _check(lib().gd_split_step(self.h, _ptr(g), _ptr(kscale), v.ctypes.data_as(_DP), float(dx),
                                   int(bool(periodic)), float(dt), int(n_steps),
                                   ctypes.byref(cnt) if count_violations else None), counted=count_violations)
        return cnt.value if count_violations else None

    def rk_advance(self, g, t, t_end, cfl, dt_max, n_substeps, kscale=None, flux_floor=0.0, count=False):
        """Per-cell steps under the CFL bound (gd_rk_advance) on g and the cell
        times t in place; with count, returns (violations, unfinished cells)."""
        _dev64(g, self.n_values, "g")
        if t is None:
            raise TypeError("t must be a float64 device tensor")
        _dev64(t, self.n_cells, "t")
        _dev64(kscale, self.n_cells, "kscale")
        v = ctypes.c_longlong(0)
        u = ctypes.c_longlong(0)
        _check(lib().gd_rk_advance(self.h, _ptr(g), _ptr(kscale), _ptr(t), float(t_end), float(cfl), float(dt_max),
                                   float(flux_floor), int(n_substeps), ctypes.byref(v) if count else None,
                                   ctypes.byref(u) if count else None), counted=count)
        return (v.value, u.value) if count else None

    def timing(self, enable=True):
        _check(lib().gd_plan_timing(self.h, int(bool(enable))))

    def rk_forward(self, g, dt, n_steps, kscale=None, count_violations=False):
        """gd_rk_step on g in place, recording checkpoints; returns (states, gammas[, violations])."""
        import torch
        _dev64(g, self.n_values, "g")
        _dev64(kscale, self.n_cells, "kscale")
        st = torch.empty((1 + 3 * n_steps) * self.n_values, dtype=torch.float64, device=g.device)
        gm = torch.empty((1 + 3 * n_steps) * self.n_bins, dtype=torch.float64, device=g.device)
        v = ctypes.c_longlong(0)
        _check(lib().gd_rk_forward(self.h, _ptr(g), _ptr(kscale), float(dt), int(n_steps), _ptr(st), _ptr(gm),
                                   ctypes.byref(v) if count_violations else None), counted=count_violations)
        return (st, gm, v.value) if count_violations else (st, gm)

    def adjoint(self, states, gammas, dt, n_steps, lam, kscale=None, want_kscale=True, want_vfrag=True):
        """lam (dLoss/dg_final) -> dLoss/dg_input in place; returns (dkscale, dvfrag)."""
        import torch
        _dev64(lam, self.n_values, "lam")
        _dev64(kscale, self.n_cells, "kscale")
        _dev64(states, (1 + 3 * n_steps) * self.n_values, "states")
        _dev64(gammas, (1 + 3 * n_steps) * self.n_bins, "gammas")
        dks = torch.empty(self.n_cells, dtype=torch.float64, device=lam.device) if want_kscale else None
        dvf = torch.empty(self.n_cells, dtype=torch.float64, device=lam.device) if want_vfrag else None
        _check(lib().gd_adjoint(self.h, _ptr(states), _ptr(gammas), _ptr(kscale), float(dt), int(n_steps),
                                _ptr(lam), _ptr(dks), _ptr(dvf)))
        return dks, dvf

    def collision_vjp(self, g, mu, kscale=None, grad=None):
        """grad += (dL/dg)^T mu; returns (grad, dkscale, dvfrag)."""
        import torch
        _dev64(g, self.n_values, "g")
        _dev64(mu, self.n_values, "mu")
        _dev64(kscale, self.n_cells, "kscale")
        if grad is None:
            grad = torch.zeros_like(g)
        _dev64(grad, self.n_values, "grad")
        dks = torch.empty(self.n_cells, dtype=torch.float64, device=g.device)
        dvf = torch.empty(self.n_cells, dtype=torch.float64, device=g.device)
        _check(lib().gd_collision_vjp(self.h, _ptr(g), _ptr(kscale), _ptr(mu), _ptr(grad), _ptr(dks), _ptr(dvf)))
        return grad, dks, dvf

    def set_variant(self, waves=4, rows=1, xcd=1, tiles_per_wave=1):
        """Contraction variant: waves per workgroup (4 or 8), tiles per wave (1 or 2), row
        blocks per item (0 = all), items grouped by XCD (1) or in one largest-first order (0)."""
        _check(lib().gd_plan_set_variant(self.h, int(waves), int(tiles_per_wave), int(rows), int(xcd)))

    def group_rows(self):
        """Row blocks per work item of every group (gd_plan_group_rows)."""
        out = (ctypes.c_int * len(self.tensors))()
        _check(lib().gd_plan_group_rows(self.h, out))
        return list(out)

    def variant(self):
        w, t, r, x, n = (ctypes.c_int() for _ in range(5))
        f = ctypes.c_double()
        _check(lib().gd_plan_variant(self.h, ctypes.byref(w), ctypes.byref(t), ctypes.byref(r), ctypes.byref(x),
                                     ctypes.byref(n), ctypes.byref(f)))
        return {"waves": w.value, "tiles_per_wave": t.value, "rows": r.value, "xcd": x.value, "n_items": n.value,
                "exec_flops": f.value}

    def algorithmic_flops(self):
        """Flops one right-hand-side evaluation of every cell must do (2 nnz of the
        folded tensor of each cell's level, plus its level-difference part)."""
        f = ctypes.c_double()
        _check(lib().gd_plan_algorithmic_flops(self.h, ctypes.byref(f)))
        return f.value

    def autotune(self, g, kscale=None, cache_path=None):
        """Time every contraction variant on state g and keep the fastest."""
        _dev64(g, self.n_values, "g")
        _dev64(kscale, self.n_cells, "kscale")
        w, t, r, x = (ctypes.c_int() for _ in range(4))
        cp = cache_path.encode() if cache_path else None
        _check(lib().gd_plan_autotune(self.h, _ptr(g), _ptr(kscale), cp, ctypes.byref(w), ctypes.byref(t),
                                      ctypes.byref(r), ctypes.byref(x)))
        return {"waves": w.value, "tiles_per_wave": t.value, "rows": r.value, "xcd": x.value}

    def checks(self):
        """The device-check word of the checked build since the last read (gd_plan_checks);
        raises GDError (GD_EUNSUPPORTED) on the regular build."""
        f = ctypes.c_uint(0)
        _check(lib().gd_plan_checks(self.h, ctypes.byref(f)))
        return f.value

    def set_lanes(self, lanes=0):
        """Lanes of gd_rk_step, gd_rk_advance and gd_collision_rhs (0 = by size): cell
        ranges stepped side by side on streams of their own (gd_plan_set_lanes)."""
        _check(lib().gd_plan_set_lanes(self.h, int(lanes)))

    def lanes(self):
        """(lanes in use, first 32-slot tile of each)."""
        n = ctypes.c_int()
        ft = (ctypes.c_int * 8)()
        _check(lib().gd_plan_lanes(self.h, ctypes.byref(n), ft))
        return n.value, list(ft[:n.value])

    def use_graph(self, enable=True):
        _check(lib().gd_plan_use_graph(self.h, int(bool(enable))))

    def contraction_time(self):
        """(total ms, launches) of the contraction kernels since timing was enabled."""
        ms = ctypes.c_double()
        n = ctypes.c_int()
        _check(lib().gd_plan_contraction_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def stage_time(self):
        """(total ms, launches) of the stage kernels since timing was enabled."""
        ms = ctypes.c_double()
        n = ctypes.c_int()
        _check(lib().gd_plan_stage_time(self.h, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and _lib is not None:
            _lib.gd_plan_destroy(h)
            self.h = None


_RKSOLVE = None


def _rksolve_class():
    global _RKSOLVE
    if _RKSOLVE is None:
        import torch

        class RKSolve(torch.autograd.Function):
            """n_steps of SSP-RK3 with the limiter (gd_rk_forward) whose backward is the
            library's adjoint (gd_adjoint): gradients for the initial state, the per-cell
            kernel scale and the per-cell fragmentation threshold.  When the threshold
            tensor's values differ from the plan's, the plan's brackets and blend weights
            are rebuilt from them first (gd_plan_set_vfrag)."""

            @staticmethod
            def forward(ctx, g0, kscale, vfrag, plan, dt, n_steps):
                if vfrag is not None:
                    v = vfrag.detach().to("cpu", torch.float64).numpy().reshape(-1)
                    if plan.vfrag is None or not np.array_equal(v, plan.vfrag):
                        plan.set_vfrag(v)
                g = g0.detach().clone().contiguous()
                ks = None if kscale is None else kscale.detach().contiguous()
                states, gammas = plan.rk_forward(g, dt, n_steps, kscale=ks)
                ctx.plan, ctx.dt, ctx.n_steps = plan, dt, n_steps
                ctx.ks = ks
                ctx.save_for_backward(states, gammas)
                return g

            @staticmethod
            def backward(ctx, grad):
                states, gammas = ctx.saved_tensors
                lam = grad.detach().to(torch.float64).clone().contiguous()
                dks, dvf = ctx.plan.adjoint(states, gammas, ctx.dt, ctx.n_steps, lam, kscale=ctx.ks,
                                            want_kscale=ctx.needs_input_grad[1],
                                            want_vfrag=ctx.needs_input_grad[2])
                return lam, dks, dvf, None, None, None

        _RKSOLVE = RKSolve
    return _RKSOLVE


def rk_solve(plan, g0, dt, n_steps, kscale=None, vfrag=None):
    """Differentiable n_steps of SSP-RK3 on the plan (see RKSolve)."""
    return _rksolve_class().apply(g0, kscale, vfrag, plan, dt, n_steps)
