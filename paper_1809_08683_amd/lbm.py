"""Thin Python binding of the C ABI in include/lbm.h (argument marshalling only).

Every step of the lattice Boltzmann path runs in the gfx950 kernels of
liblbm_hip.so; this module only converts case dicts (see ``inputs``) into
the C parameter blocks and numpy arrays into pointers.  It raises
``LibraryMissing`` when the HIP library is not built: there is no fallback.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_hip.so")

OK, EINVAL, ENOMEM, EDEVICE, EDIVERGED, ESTATE = 0, -1, -2, -3, -4, -5
EOS = {"decoupled": 0, "ideal": 1, "vdw": 2, "cs": 3}
VISC = {"const": 0, "linear": 1, "sutherland": 2}
PREC = {"f64": 0, "f32": 1, "f16s": 2, "f32g16": 3}


class LibraryMissing(RuntimeError):
    pass


class LBMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


class Diverged(LBMError):
    pass


class Eos(C.Structure):
    _fields_ = [("kind", C.c_int), ("R", C.c_double), ("rho0", C.c_double), ("T0", C.c_double),
                ("a", C.c_double), ("b", C.c_double)]


class Relax(C.Structure):
    _fields_ = [("nu0", C.c_double), ("bulk_ratio", C.c_double), ("law", C.c_int),
                ("sutherland_S", C.c_double)]


class Side(C.Structure):
    _fields_ = [("wall", C.c_int), ("ux", C.c_double), ("uy", C.c_double), ("adiabatic", C.c_int),
                ("T", C.c_double)]


class Boundary(C.Structure):
    _fields_ = [("side", Side * 4), ("extrap_order", C.c_int)]


class Options(C.Structure):
    _fields_ = [("fx", C.c_double), ("fy", C.c_double), ("per_mass", C.c_int), ("prec", C.c_int),
                ("cubic", C.c_int), ("cp", C.c_double), ("cv_rule", C.c_int), ("seg_rows", C.c_int),
                ("hip_stream", C.c_void_p)]


class TuneResult(C.Structure):
    _fields_ = [("variant", C.c_int), ("xw_scale", C.c_double), ("bands_per_xcd", C.c_int),
                ("ms_per_step", C.c_double), ("default_ms_per_step", C.c_double), ("trials", C.c_int),
                ("from_cache", C.c_int)]


STEP_GRAPH = 1
STEP_PERSISTENT = 2
TUNE_CACHE = os.path.join(_HERE, "tune_cache.json")

_lib = None
_D = C.POINTER(C.c_double)


def load_library():
    """Load liblbm_hip.so (built by ``paper_1809_08683_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise LibraryMissing(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    try:
        # PyTorch ships its own HIP runtime with the same soname; loading it
        # first makes this library bind to that one copy instead of a second
        # runtime that would then see no device.
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(LIB_PATH)
    vp, cp = C.c_void_p, C.POINTER(C.c_void_p)
    sig = {
        "lbm_create": ([C.c_int, C.c_int, C.POINTER(Eos), C.c_double, C.c_double, C.POINTER(Relax),
                        C.POINTER(Boundary), C.POINTER(Options), cp], C.c_int),
        "lbm_workspace_bytes": ([C.c_int, C.c_int, C.c_int], C.c_size_t),
        "lbm_create_ex": ([C.c_int, C.c_int, C.POINTER(Eos), C.c_double, C.c_double, C.POINTER(Relax),
                           C.POINTER(Boundary), C.POINTER(Options), vp, C.c_size_t, cp], C.c_int),
        "lbm_init": ([vp, _D, _D, _D, _D], C.c_int),
        "lbm_step": ([vp, C.c_longlong], C.c_int),
        "lbm_step_timed": ([vp, C.c_longlong, _D], C.c_int),
        "lbm_step_ex": ([vp, C.c_longlong, C.c_int, _D], C.c_int),
        "lbm_case_diverged_at": ([vp, C.c_int], C.c_longlong),
        "lbm_set_launch_config": ([vp, C.c_int, C.c_double, C.c_int], C.c_int),
        "lbm_set_persistent_spin_limit": ([vp, C.c_uint], C.c_int),
        "lbm_autotune": ([vp, C.c_int, C.c_char_p, C.POINTER(TuneResult)], C.c_int),
        "lbm_macros": ([vp, _D, _D, _D, _D, _D], C.c_int),
        "lbm_nusselt": ([vp, C.c_int, _D], C.c_int),
        "lbm_totals": ([vp, _D, _D, _D, _D], C.c_int),
        "lbm_state_bytes": ([vp], C.c_size_t),
        "lbm_save": ([vp, vp, C.c_size_t], C.c_int),
        "lbm_load": ([vp, vp, C.c_size_t], C.c_int),
        "lbm_time": ([vp], C.c_longlong),
        "lbm_last_error": ([vp], C.c_char_p),
        "lbm_destroy": ([vp], None),
        "lbm_batch_create": ([C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_int), C.POINTER(Eos),
                              _D, _D, C.POINTER(Relax), C.POINTER(Boundary), C.POINTER(Options), cp], C.c_int),
        "lbm_batch_size": ([vp], C.c_int),
        "lbm_case_init": ([vp, C.c_int, _D, _D, _D, _D], C.c_int),
        "lbm_case_init_static": ([vp, C.c_int, _D, _D, _D, _D], C.c_int),
        "lbm_case_macros": ([vp, C.c_int, _D, _D, _D, _D, _D], C.c_int),
        "lbm_case_nusselt": ([vp, C.c_int, C.c_int, _D], C.c_int),
        "lbm_case_totals": ([vp, C.c_int, _D, _D, _D, _D], C.c_int),
        "lbm_batch_flags": ([vp, C.POINTER(C.c_int)], C.c_int),
        "lbm_batch_step": ([vp, C.c_longlong], C.c_int),
        "lbm_batch_nusselt": ([vp, C.c_int, _D, C.POINTER(C.c_int)], C.c_int),
        "lbm_work_items": ([vp], C.c_longlong),
        "lbm_copy_bandwidth": ([C.c_size_t, C.c_int, vp, _D, _D], C.c_int),
        "lbm_rounding_operand": ([C.c_int, C.c_int, C.c_int, C.c_uint, C.c_int], C.c_uint),
        "lbm_round_half_stochastic": ([C.c_float, C.c_uint], C.c_double),
        "lbm_round_half_device": ([vp, vp, vp, C.c_longlong, vp], C.c_int),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def exported_symbols():
    """Names of the C ABI entry points this binding calls."""
    return ["lbm_create", "lbm_workspace_bytes", "lbm_create_ex", "lbm_init", "lbm_step",
            "lbm_step_timed", "lbm_step_ex", "lbm_case_diverged_at", "lbm_set_launch_config",
            "lbm_set_persistent_spin_limit", "lbm_autotune", "lbm_macros", "lbm_nusselt", "lbm_totals", "lbm_state_bytes",
            "lbm_save", "lbm_load", "lbm_time", "lbm_last_error", "lbm_destroy",
            "lbm_batch_create", "lbm_batch_size", "lbm_case_init", "lbm_case_init_static", "lbm_case_macros",
            "lbm_case_nusselt", "lbm_case_totals", "lbm_batch_flags", "lbm_batch_step", "lbm_batch_nusselt", "lbm_work_items",
            "lbm_copy_bandwidth", "lbm_rounding_operand", "lbm_round_half_stochastic", "lbm_round_half_device"]


def copy_bandwidth(nbytes: int, iters: int = 20, stream=None):
    """Measured device copy bandwidth (GB/s) and ms per copy of ``nbytes``."""
    lib = load_library()
    g, ms = C.c_double(), C.c_double()
    rc = lib.lbm_copy_bandwidth(int(nbytes), int(iters), _stream_handle(stream), C.byref(g), C.byref(ms))
    if rc != OK:
        raise LBMError(rc, "lbm_copy_bandwidth")
    return g.value, ms.value


def rounding_operand(prec, x: int, y: int, t: int, q: int) -> int:
    """32-bit random operand of the stochastic rounding of DF row q at node
    (x, y) in step t (host computation with the kernels' code)."""
    return int(load_library().lbm_rounding_operand(PREC[prec] if isinstance(prec, str) else int(prec),
                                                    int(x), int(y), int(t) & 0xFFFFFFFF, int(q)))


def round_half_stochastic(v: float, r: int) -> float:
    """The library's host model of the device's stochastic FP16 rounding."""
    return float(load_library().lbm_round_half_stochastic(float(v), int(r) & 0xFFFFFFFF))


def round_half_device(v, r, stream=None):
    """Stochastic FP16 rounding on the device with the store codec's code:
    v (float32) and r (int32 bit patterns) are device tensors of equal
    length; returns the FP16 values as a float32 device tensor."""
    import torch
    if v.dtype != torch.float32 or r.dtype != torch.int32 or v.numel() != r.numel():
        raise ValueError("v must be float32 and r int32 of the same length")
    v, r = v.contiguous(), r.contiguous()
    out = torch.empty_like(v)
    rc = load_library().lbm_round_half_device(v.data_ptr(), r.data_ptr(), out.data_ptr(), v.numel(),
                                              _stream_handle(stream))
    if rc != OK:
        raise LBMError(rc, "lbm_round_half_device")
    return out


def _ptr(a):
    return None if a is None else a.ctypes.data_as(_D)


def param_blocks(case: dict, stream=None, seg_rows=0):
    """C parameter blocks (Eos, Relax, Boundary, Options) of a case dict."""
    e = Eos(EOS[case.get("eos", "ideal")], float(case.get("R", 0.0)), float(case.get("rho0", 1.0)),
            float(case.get("T0", 1.0)), float(case.get("a", 0.0)), float(case.get("b", 0.0)))
    r = Relax(float(case["nu0"]), float(case.get("bulk_ratio", 1.0)), VISC[case.get("visc_law", "const")],
              float(case.get("suth_S", 0.0)))
    b = Boundary()
    for s in range(4):
        sd = case["sides"][s]
        u = sd.get("u", (0.0, 0.0))
        b.side[s] = Side(1 if sd["kind"] == "wall" else 0, float(u[0]), float(u[1]),
                         1 if sd.get("thermal", "dirichlet") == "adiabatic" else 0,
                         float(sd.get("T", case.get("T0", 1.0))))
    b.extrap_order = int(case.get("extrap_order", 2))
    fx, fy = case.get("force", (0.0, 0.0))
    o = Options(float(fx), float(fy), int(bool(case.get("per_mass", False))), PREC[case.get("prec", "f32")],
                int(case.get("cubic", 2)), float(case.get("cp", 0.0)), int(case.get("cv_rule", 0)),
                int(seg_rows or case.get("seg_rows", 0)), stream)
    return e, r, b, o


def _stream_handle(stream):
    if stream is None:
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


class _Base:
    def __init__(self):
        self.lib = load_library()
        self.h = C.c_void_p()
        self.diverged = False

    def _check(self, rc, what):
        if rc == OK:
            return
        msg = self.lib.lbm_last_error(self.h).decode() if self.h else what
        if rc == EDIVERGED:
            raise Diverged(rc, f"{what}: {msg}")
        raise LBMError(rc, f"{what}: {msg}")

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            self.lib.lbm_destroy(self.h)
            self.h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, n: int = 1):
        self._check(self.lib.lbm_step(self.h, int(n)), "lbm_step")
        return self

    def step_timed(self, n: int, allow_diverged: bool = False) -> float:
        """Advance n steps; return their device time (ms).  With
        allow_diverged a divergence is recorded in ``self.diverged`` instead
        of raised."""
        ms = C.c_double(0.0)
        rc = self.lib.lbm_step_timed(self.h, int(n), C.byref(ms))
        self.diverged = rc == EDIVERGED
        if not (rc == EDIVERGED and allow_diverged):
            self._check(rc, "lbm_step_timed")
        return ms.value

    def step_ex(self, n: int, graph: bool = False, allow_diverged: bool = False, persistent: bool = False) -> float:
        """Advance n steps (as one replayed HIP graph if ``graph``; in one
        launch of the persistent kernel if ``persistent``); return their
        device time (ms)."""
        ms = C.c_double(0.0)
        flags = (STEP_GRAPH if graph else 0) | (STEP_PERSISTENT if persistent else 0)
        rc = self.lib.lbm_step_ex(self.h, int(n), flags, C.byref(ms))
        self.diverged = rc == EDIVERGED
        if not (rc == EDIVERGED and allow_diverged):
            self._check(rc, "lbm_step_ex")
        return ms.value

    def set_persistent_spin_limit(self, polls: int):
        self._check(self.lib.lbm_set_persistent_spin_limit(self.h, int(polls)), "lbm_set_persistent_spin_limit")
        return self

    def diverged_at(self, k: int = 0) -> int:
        return int(self.lib.lbm_case_diverged_at(self.h, int(k)))

    def set_launch_config(self, variant: int = 0, xw_scale: float = 1.0, bands_per_xcd: int = 4):
        self._check(self.lib.lbm_set_launch_config(self.h, int(variant), float(xw_scale), int(bands_per_xcd)),
                    "lbm_set_launch_config")
        return self

    def autotune(self, trial_steps: int = 0, cache_path=TUNE_CACHE) -> dict:
        """Launch-configuration autotuner (see lbm_autotune); cache_path None
        tunes without reading or writing a cache."""
        r = TuneResult()
        path = None if cache_path is None else os.fsencode(cache_path)
        self._check(self.lib.lbm_autotune(self.h, int(trial_steps), path, C.byref(r)), "lbm_autotune")
        return {n: getattr(r, n) for n, _ in TuneResult._fields_}

    @property
    def time(self) -> int:
        return int(self.lib.lbm_time(self.h))

    @property
    def work_items(self) -> int:
        return int(self.lib.lbm_work_items(self.h))

    def save(self) -> bytes:
        n = self.lib.lbm_state_bytes(self.h)
        buf = (C.c_char * n)()
        self._check(self.lib.lbm_save(self.h, buf, n), "lbm_save")
        return bytes(buf)

    def load(self, blob: bytes):
        buf = C.create_string_buffer(blob, len(blob))
        self._check(self.lib.lbm_load(self.h, buf, len(blob)), "lbm_load")
        return self


class Context(_Base):
    """One lattice on the GPU.  ``workspace="torch"`` places the device arrays
    in a torch tensor (PyTorch as the allocator); ``stream`` is a torch
    stream or a raw hipStream_t."""

    def __init__(self, case: dict, stream=None, workspace=None, seg_rows=0):
        super().__init__()
        self.case = dict(case)
        self.nx, self.ny = int(case["nx"]), int(case["ny"])
        self._blocks = param_blocks(case, _stream_handle(stream), seg_rows)
        e, r, b, o = self._blocks
        self._ws = None
        if workspace == "torch":
            import torch
            nbytes = self.lib.lbm_workspace_bytes(self.nx, self.ny, o.prec)
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
            rc = self.lib.lbm_create_ex(self.nx, self.ny, C.byref(e), float(case["Pr"]), float(case["gamma"]),
                                        C.byref(r), C.byref(b), C.byref(o), C.c_void_p(self._ws.data_ptr()),
                                        nbytes, C.byref(self.h))
        else:
            rc = self.lib.lbm_create(self.nx, self.ny, C.byref(e), float(case["Pr"]), float(case["gamma"]),
                                     C.byref(r), C.byref(b), C.byref(o), C.byref(self.h))
        if rc != OK:
            msg = self.lib.lbm_last_error(self.h).decode() if self.h.value else "create failed"
            self.close()
            raise LBMError(rc, f"lbm_create: {msg}")

    def init(self, rho=None, ux=None, uy=None, T=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
                for a in (rho, ux, uy, T)]
        for a in arrs:
            if a is not None and a.size != self.nx * self.ny:
                raise ValueError("initial field has the wrong size")
        self._check(self.lib.lbm_init(self.h, *[_ptr(a) for a in arrs]), "lbm_init")
        return self

    def init_static(self, rho=None, ux=None, uy=None, T=None):
        """As init, through the entry point that stages the fields in the
        library's static device scratch (no device allocation)."""
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
                for a in (rho, ux, uy, T)]
        for a in arrs:
            if a is not None and a.size != self.nx * self.ny:
                raise ValueError("initial field has the wrong size")
        self._check(self.lib.lbm_case_init_static(self.h, 0, *[_ptr(a) for a in arrs]), "lbm_case_init_static")
        return self

    def macros(self) -> dict:
        nn = self.nx * self.ny
        out = {k: np.empty(nn) for k in ("rho", "ux", "uy", "T", "p")}
        self._check(self.lib.lbm_macros(self.h, *[_ptr(out[k]) for k in ("rho", "ux", "uy", "T", "p")]),
                    "lbm_macros")
        return {k: v.reshape(self.ny, self.nx) for k, v in out.items()}

    def nusselt(self, side: int = 0) -> float:
        v = C.c_double()
        self._check(self.lib.lbm_nusselt(self.h, int(side), C.byref(v)), "lbm_nusselt")
        return v.value

    def totals(self):
        v = [C.c_double() for _ in range(4)]
        self._check(self.lib.lbm_totals(self.h, *[C.byref(x) for x in v]), "lbm_totals")
        return tuple(x.value for x in v)


class Batch(_Base):
    """Many independent lattices stepped together (one launch per step)."""

    def __init__(self, cases: list, stream=None, seg_rows=0):
        super().__init__()
        n = len(cases)
        self.cases = [dict(c) for c in cases]
        blocks = [param_blocks(c, _stream_handle(stream), seg_rows) for c in cases]
        nx = (C.c_int * n)(*[int(c["nx"]) for c in cases])
        ny = (C.c_int * n)(*[int(c["ny"]) for c in cases])
        E = (Eos * n)(*[b[0] for b in blocks])
        R = (Relax * n)(*[b[1] for b in blocks])
        B = (Boundary * n)(*[b[2] for b in blocks])
        O = (Options * n)(*[b[3] for b in blocks])
        Pr = np.array([float(c["Pr"]) for c in cases])
        G = np.array([float(c["gamma"]) for c in cases])
        rc = self.lib.lbm_batch_create(n, nx, ny, E, _ptr(Pr), _ptr(G), R, B, O, C.byref(self.h))
        if rc != OK:
            msg = self.lib.lbm_last_error(self.h).decode() if self.h.value else "create failed"
            self.close()
            raise LBMError(rc, f"lbm_batch_create: {msg}")

    def __len__(self):
        return len(self.cases)

    def init(self, k: int, rho=None, ux=None, uy=None, T=None):
        arrs = [None if a is None else np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
                for a in (rho, ux, uy, T)]
        self._check(self.lib.lbm_case_init(self.h, int(k), *[_ptr(a) for a in arrs]), "lbm_case_init")
        return self

    def macros(self, k: int) -> dict:
        nx, ny = int(self.cases[k]["nx"]), int(self.cases[k]["ny"])
        out = {f: np.empty(nx * ny) for f in ("rho", "ux", "uy", "T", "p")}
        self._check(self.lib.lbm_case_macros(self.h, int(k), *[_ptr(out[f]) for f in ("rho", "ux", "uy", "T", "p")]),
                    "lbm_case_macros")
        return {f: v.reshape(ny, nx) for f, v in out.items()}

    def nusselt(self, k: int, side: int = 0) -> float:
        v = C.c_double()
        self._check(self.lib.lbm_case_nusselt(self.h, int(k), int(side), C.byref(v)), "lbm_case_nusselt")
        return v.value

    def totals(self, k: int):
        v = [C.c_double() for _ in range(4)]
        self._check(self.lib.lbm_case_totals(self.h, int(k), *[C.byref(x) for x in v]), "lbm_case_totals")
        return tuple(x.value for x in v)

    def batch_step(self, n: int):
        """Advance every case n steps; divergence is reported per case."""
        self._check(self.lib.lbm_batch_step(self.h, int(n)), "lbm_batch_step")
        return self

    def batch_nusselt(self, side: int = 0):
        """(nu, diverged) of every case."""
        n = len(self.cases)
        nu = np.empty(n)
        dv = (C.c_int * n)()
        self._check(self.lib.lbm_batch_nusselt(self.h, int(side), _ptr(nu), dv), "lbm_batch_nusselt")
        return nu, list(dv)

    def flags(self):
        out = (C.c_int * len(self.cases))()
        self._check(self.lib.lbm_batch_flags(self.h, out), "lbm_batch_flags")
        return list(out)

    def step(self, n: int = 1, allow_diverged: bool = False):
        rc = self.lib.lbm_step(self.h, int(n))
        if rc == EDIVERGED and allow_diverged:
            return self
        self._check(rc, "lbm_step")
        return self
