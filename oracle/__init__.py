"""FP64 CPU oracle for the three coupled D2Q9 lattice Boltzmann equations of
Wang, He & Wang, "Phase-field-based lattice Boltzmann model for simulating
thermocapillary flows" (arXiv:2306.11320), Sec. 3 and Sec. 4.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package.  It shares no code with the HIP path:
the C source ``lbm_oracle.c`` is compiled here with gcc, and this module only
marshals arguments into it through ctypes.

Parity status of each function is stated in its docstring; the pins that check
the oracle against what the paper and the mathematics fix live in
``tests/test_oracle_*.py``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
_lock = threading.Lock()
_lib = None

PERIODIC, WALL_T, WALL_ADIABATIC, INLET, OUTLET = 0, 1, 2, 3, 4


def build() -> str:
    """Compile the oracle with gcc (plain FP64, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c99", "-Wall", "-Wextra", "-Wno-unused-parameter", _SRC, "-o", _LIB + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("bc", C.c_int32 * 4), ("grad_mode", C.c_int32),
        ("n_bubbles", C.c_int32), ("collision", C.c_int32), ("force_form", C.c_int32), ("trt_magic", C.c_double),
        ("rho_l", C.c_double), ("rho_h", C.c_double), ("mu_l", C.c_double), ("mu_h", C.c_double),
        ("lam_l", C.c_double), ("lam_h", C.c_double), ("rcp_l", C.c_double), ("rcp_h", C.c_double),
        ("sigma_ref", C.c_double), ("sigma_T", C.c_double), ("sigma_TT", C.c_double), ("T_ref", C.c_double),
        ("W", C.c_double), ("M", C.c_double), ("Gx", C.c_double), ("Gy", C.c_double),
        ("tw_mean", C.c_double * 4), ("tw_amp", C.c_double * 4), ("tw_k", C.c_double * 4),
        ("tw_slope", C.c_double * 4),
        ("u_in", C.c_double), ("phi_in", C.c_double), ("T_in", C.c_double),
        ("bubble_x", C.c_double * 4), ("bubble_y", C.c_double * 4),
    ]


class Diag(C.Structure):
    _fields_ = [
        ("step", C.c_int64), ("mass_phi", C.c_double), ("vol_light", C.c_double), ("heat", C.c_double),
        ("sum_neg", C.c_double), ("u_r", C.c_double), ("ux_r", C.c_double), ("xc", C.c_double),
        ("yc", C.c_double), ("max_u", C.c_double), ("n_nonfinite", C.c_int64), ("n_neg", C.c_int64),
        ("bub_x", C.c_double * 4), ("bub_y", C.c_double * 4), ("bub_ux", C.c_double * 4),
        ("bub_uy", C.c_double * 4), ("bub_sum", C.c_double * 4),
    ]

    def as_dict(self) -> dict:
        out = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            out[name] = list(v) if isinstance(v, C.Array) else v
        return out


def _bind(L):
    """Declares the C signatures of an oracle library handle."""
    dp = C.POINTER(C.c_double)
    L.orc_create.restype = C.c_void_p
    L.orc_create.argtypes = [C.POINTER(Params), dp, dp, dp, dp]
    L.orc_destroy.argtypes = [C.c_void_p]
    L.orc_step.argtypes = [C.c_void_p, C.c_int64]
    L.orc_fields.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
    L.orc_macros_all.argtypes = [C.c_void_p, dp]
    L.orc_get_state.argtypes = [C.c_void_p, dp, dp, dp, dp, C.POINTER(C.c_int64)]
    L.orc_set_state.argtypes = [C.c_void_p, dp, dp, dp, dp, C.c_int64]
    L.orc_diagnostics.argtypes = [C.c_void_p, C.POINTER(Diag)]
    L.orc_set_threads.argtypes = [C.c_int]
    L.orc_step_count_writes.argtypes = [C.c_void_p, C.POINTER(C.c_int)]
    L.orc_get_threads.restype = C.c_int
    assert L.orc_sizeof_params() == C.sizeof(Params), "oracle params layout mismatch"
    assert L.orc_sizeof_diag() == C.sizeof(Diag), "oracle diag layout mismatch"
    return L


def lib():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
                build()
            _lib = _bind(C.CDLL(_LIB))
    return _lib


def build_variant(source_text: str, out_path: str) -> str:
    """Compiles an edited copy of the oracle's C source (same flags) into
    out_path.  Used by the tests that plant a mistake in the oracle to show
    that its pins catch it; the product never calls this."""
    src = out_path + ".c"
    with open(src, "w") as fh:
        fh.write(source_text)
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
           "-std=c99", "-w", src, "-o", out_path, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


class use_library:
    """Context manager: Oracle objects created inside it run the library at
    `path` (an oracle variant built by build_variant)."""

    def __init__(self, path: str):
        self.path = path

    def __enter__(self):
        global _lib
        lib()
        with _lock:
            self._saved = _lib
            _lib = _bind(C.CDLL(self.path))
        return self

    def __exit__(self, *exc):
        global _lib
        with _lock:
            _lib = self._saved
        return False


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_params(cfg: dict) -> Params:
    """Marshal a workload parameter dict (see ``paper_2306_11320_amd.workloads``)."""
    p = Params()
    p.nx, p.ny = int(cfg["nx"]), int(cfg["ny"])
    for s in range(4):
        p.bc[s] = int(cfg["bc"][s])
        p.tw_mean[s] = float(cfg.get("tw_mean", [0.0] * 4)[s])
        p.tw_amp[s] = float(cfg.get("tw_amp", [0.0] * 4)[s])
        p.tw_k[s] = float(cfg.get("tw_k", [0.0] * 4)[s])
        p.tw_slope[s] = float(cfg.get("tw_slope", [0.0] * 4)[s])
    p.grad_mode = int(cfg.get("grad_mode", 0))
    p.collision = int(cfg.get("collision", 0))
    p.force_form = int(cfg.get("force_form", 0))
    p.trt_magic = float(cfg.get("trt_magic", 0.1875))
    bx = list(cfg.get("bubbles_x", []))
    by = list(cfg.get("bubbles_y", []))
    p.n_bubbles = len(bx)
    for b in range(len(bx)):
        p.bubble_x[b] = float(bx[b])
        p.bubble_y[b] = float(by[b])
    for k in ("rho_l", "rho_h", "mu_l", "mu_h", "sigma_ref", "sigma_T", "sigma_TT", "T_ref", "W", "Gx", "Gy",
              "phi_in", "T_in"):
        setattr(p, k, float(cfg.get(k, 0.0)))
    p.lam_l, p.lam_h = float(cfg["lambda_l"]), float(cfg["lambda_h"])
    p.rcp_l, p.rcp_h = float(cfg["rhocp_l"]), float(cfg["rhocp_h"])
    p.M = float(cfg["mobility"])
    p.u_in = float(cfg.get("u_in_mean", 0.0))
    return p


class Oracle:
    """One lattice advanced by the CPU oracle.

    ``fields0`` is a dict of host arrays ``phi, ux, uy, T`` of shape (ny, nx).
    """

    def __init__(self, cfg: dict, fields0: dict, threads: int | None = None):
        self.L = lib()
        if threads is not None:
            self.L.orc_set_threads(int(threads))
        self.cfg = cfg
        self.nx, self.ny = int(cfg["nx"]), int(cfg["ny"])
        self.params = make_params(cfg)
        arrs = [np.ascontiguousarray(fields0[k], dtype=np.float64).reshape(-1) for k in ("phi", "ux", "uy", "T")]
        for a in arrs:
            if a.size != self.nx * self.ny:
                raise ValueError("initial field has the wrong size")
        self._h = self.L.orc_create(C.byref(self.params), *[_dp(a) for a in arrs])
        if not self._h:
            raise ValueError("oracle rejected the parameters")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self.L.orc_destroy(h)
            self._h = None

    @staticmethod
    def threads() -> int:
        return lib().orc_get_threads()

    def step(self, n: int = 1) -> None:
        self.L.orc_step(self._h, int(n))

    def step_count_writes(self) -> np.ndarray:
        """One step; returns how often each slot (9, ny, nx) of the new time
        level was stored (coverage check of the streaming and boundary rules)."""
        cnt = np.zeros(9 * self.nx * self.ny, dtype=np.int32)
        if self.L.orc_step_count_writes(self._h, cnt.ctypes.data_as(C.POINTER(C.c_int))) != 0:
            raise MemoryError("oracle: out of memory")
        return cnt.reshape(9, self.ny, self.nx)

    def fields(self) -> dict:
        n = self.nx * self.ny
        out = {k: np.empty(n) for k in ("phi", "ux", "uy", "T", "p")}
        self.L.orc_fields(self._h, *[_dp(out[k]) for k in ("phi", "ux", "uy", "T", "p")])
        return {k: v.reshape(self.ny, self.nx) for k, v in out.items()}

    MACRO_NAMES = ("phi", "T", "ux", "uy", "p", "Fx", "Fy", "dphix", "dphiy", "lapphi", "dTx", "dTy", "jy")

    def macros_all(self) -> dict:
        n = self.nx * self.ny
        buf = np.empty(13 * n)
        self.L.orc_macros_all(self._h, _dp(buf))
        return {k: buf[q * n:(q + 1) * n].reshape(self.ny, self.nx) for q, k in enumerate(self.MACRO_NAMES)}

    def get_state(self) -> dict:
        n = self.nx * self.ny
        f, g, h, jp = np.empty(9 * n), np.empty(9 * n), np.empty(9 * n), np.empty(2 * n)
        st = C.c_int64(0)
        self.L.orc_get_state(self._h, _dp(f), _dp(g), _dp(h), _dp(jp), C.byref(st))
        shp = (9, self.ny, self.nx)
        return {"f": f.reshape(shp), "g": g.reshape(shp), "h": h.reshape(shp),
                "jprev": jp.reshape(2, self.ny, self.nx), "step": st.value}

    def set_state(self, f=None, g=None, h=None, jprev=None, step: int = 0) -> None:
        def conv(a):
            if a is None:
                return None, None
            a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
            return a, _dp(a)
        keep = [conv(a) for a in (f, g, h, jprev)]
        self.L.orc_set_state(self._h, *[k[1] for k in keep], int(step))

    def diagnostics(self) -> dict:
        d = Diag()
        self.L.orc_diagnostics(self._h, C.byref(d))
        return d.as_dict()
