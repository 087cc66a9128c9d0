"""ctypes wrapper of the FP64 CPU oracle (``liblbm_oracle.so``).

TEST INFRASTRUCTURE ONLY: the test-suite, the package smoke check and the
benchmark's CPU-baseline leg use it to check the GPU library.  It imports
nothing from the GPU package; cases are plain dicts of lattice-unit
parameters (see the keys of ``_FIELDS``).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm_oracle.so")

NDIAG = 14
DIAG_NAMES = ("mass_phi", "mass_psi", "xc", "yc", "ux", "uy", "p_in", "p_out",
              "phi_min", "phi_max", "psi_min", "psi_max", "nonfinite", "step")
FIELD_NAMES = ("phi", "p", "ux", "uy", "T", "psi")
INTERMEDIATE_NAMES = ("dphi_dx", "dphi_dy", "kappa", "sigma", "Fs_x", "Fs_y", "Fp_x", "Fp_y",
                      "R_x", "R_y", "omega_nu", "p_star")


class OrcCase(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("wall", C.c_int32 * 4), ("t_bc", C.c_int32 * 4), ("psi_bc", C.c_int32 * 4),
        ("psi_w", C.c_double * 4),
        ("T0", C.c_double), ("gradT", C.c_double), ("xT0", C.c_double),
        ("sigma_law", C.c_int32), ("init_kind", C.c_int32),
        ("sigma0", C.c_double), ("sigma_T", C.c_double), ("sigma_TT", C.c_double),
        ("T_ref", C.c_double), ("beta_s", C.c_double), ("psi_inf", C.c_double),
        ("rho_A", C.c_double), ("rho_B", C.c_double), ("nu_A", C.c_double), ("nu_B", C.c_double),
        ("alpha_A", C.c_double), ("alpha_B", C.c_double), ("D_psi", C.c_double),
        ("M_phi", C.c_double), ("W", C.c_double),
        ("s_lam", C.c_double), ("w_lam", C.c_double),
        ("Fext_x", C.c_double), ("Fext_y", C.c_double), ("gravity", C.c_double),
        ("xc", C.c_double), ("yc", C.c_double), ("R", C.c_double),
        ("psi_bulk", C.c_double), ("psi_band", C.c_double), ("psi_gradx", C.c_double), ("phi_noise", C.c_double),
        ("p_jump", C.c_double), ("seed", C.c_uint64),
    ]


_ARRAY_KEYS = ("wall", "t_bc", "psi_bc", "psi_w")


def make_case(params: dict) -> OrcCase:
    c = OrcCase()
    for name, _ in OrcCase._fields_:
        if name not in params:
            raise KeyError(f"oracle case is missing '{name}'")
        v = params[name]
        if name in _ARRAY_KEYS:
            arr = getattr(c, name)
            for k in range(4):
                arr[k] = v[k]
        else:
            setattr(c, name, v)
    return c


def build(force: bool = False) -> str:
    src = os.path.join(HERE, "lbm_oracle.c")
    if force or not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(src):
        subprocess.run(["make", "-s", "-B", "-C", HERE], check=True)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB_PATH)
        dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(OrcCase)]
        L.orc_free.argtypes = [C.c_void_p]
        L.orc_error.restype = C.c_char_p
        L.orc_load_fields.argtypes = [C.c_void_p, dp, dp, dp]
        L.orc_step.argtypes = [C.c_void_p, C.c_int64]
        L.orc_steps_done.restype = C.c_int64
        L.orc_steps_done.argtypes = [C.c_void_p]
        L.orc_fields.argtypes = [C.c_void_p, dp]
        L.orc_intermediates.argtypes = [C.c_void_p, dp]
        L.orc_get_populations.argtypes = [C.c_void_p, dp]
        L.orc_set_populations.argtypes = [C.c_void_p, dp]
        L.orc_diag.argtypes = [C.c_void_p, dp]
        L.orc_threads.restype = C.c_int
        L.orc_matrix_P.argtypes = [dp]
        L.orc_matrix_Pinv.argtypes = [dp]
        L.orc_matrix_F.argtypes = [C.c_double, C.c_double, dp]
        L.orc_matrix_Finv.argtypes = [C.c_double, C.c_double, dp]
        L.orc_eq_g.argtypes = [C.c_double] * 4 + [dp]
        L.orc_source_g.argtypes = [C.c_double] * 6 + [dp]
        L.orc_collide_g.argtypes = [dp] + [C.c_double] * 9 + [dp]
        L.orc_collide_ad.argtypes = [dp] + [C.c_double] * 6 + [dp]
        L.orc_stream_only.argtypes = [C.c_void_p, dp, dp]
        L.orc_splitmix64.restype = C.c_uint64
        L.orc_splitmix64.argtypes = [C.c_uint64, C.c_uint64]
        L.orc_grad_periodic.argtypes = [dp, C.c_int32, C.c_int32, dp, dp]
        _lib = L
    return _lib


def threads() -> int:
    return int(lib().orc_threads())


class Oracle:
    """One lattice (one case) advanced by the FP64 oracle."""

    def __init__(self, params: dict):
        self.params = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        self._c = make_case(params)
        h = lib().orc_create(C.byref(self._c))
        if not h:
            raise ValueError(lib().orc_error().decode())
        self._h = h

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            lib().orc_free(h)
            self._h = None

    @property
    def step_count(self) -> int:
        return int(lib().orc_steps_done(self._h))

    def step(self, n: int = 1):
        lib().orc_step(self._h, int(n))
        return self

    def load_fields(self, phi, T, psi):
        shp = (self.ny, self.nx)
        a = [np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), shp)) for v in (phi, T, psi)]
        lib().orc_load_fields(self._h, *a)

    def fields(self) -> dict:
        out = np.empty((6, self.ny, self.nx))
        lib().orc_fields(self._h, out)
        return {k: out[i] for i, k in enumerate(FIELD_NAMES)}

    def intermediates(self) -> dict:
        out = np.empty((12, self.ny, self.nx))
        lib().orc_intermediates(self._h, out)
        return {k: out[i] for i, k in enumerate(INTERMEDIATE_NAMES)}

    def populations(self) -> np.ndarray:
        out = np.empty((4, 9, self.ny, self.nx))
        lib().orc_get_populations(self._h, out)
        return out

    def set_populations(self, pops: np.ndarray):
        lib().orc_set_populations(self._h, np.ascontiguousarray(pops, dtype=np.float64))

    def stream_only(self, post: np.ndarray) -> np.ndarray:
        """Stream given post-collision populations [4][9][ny][nx] with the
        wall rules; returns the streamed populations."""
        out = np.empty((4, 9, self.ny, self.nx))
        lib().orc_stream_only(self._h, np.ascontiguousarray(post, dtype=np.float64), out)
        return out

    def diag(self) -> dict:
        out = np.empty(NDIAG)
        lib().orc_diag(self._h, out)
        return {k: float(out[i]) for i, k in enumerate(DIAG_NAMES)}


# ---- unit pieces -----------------------------------------------------------------

def matrix_P():
    out = np.empty(81)
    lib().orc_matrix_P(out)
    return out.reshape(9, 9)


def matrix_Pinv():
    out = np.empty(81)
    lib().orc_matrix_Pinv(out)
    return out.reshape(9, 9)


def matrix_F(ux, uy):
    out = np.empty(81)
    lib().orc_matrix_F(ux, uy, out)
    return out.reshape(9, 9)


def matrix_Finv(ux, uy):
    out = np.empty(81)
    lib().orc_matrix_Finv(ux, uy, out)
    return out.reshape(9, 9)


def eq_g(p, rho, ux, uy):
    out = np.empty(9)
    lib().orc_eq_g(p, rho, ux, uy, out)
    return out


def source_g(Ftx, Fty, Fpx, Fpy, ux, uy):
    out = np.empty(9)
    lib().orc_source_g(Ftx, Fty, Fpx, Fpy, ux, uy, out)
    return out


def collide_g(g, p, rho, ux, uy, Ftx, Fty, Fpx, Fpy, omega_nu):
    out = np.empty(9)
    lib().orc_collide_g(np.ascontiguousarray(g, dtype=np.float64), p, rho, ux, uy, Ftx, Fty, Fpx, Fpy,
                        omega_nu, out)
    return out


def collide_ad(pop, X, jx, jy, omega1, ux, uy):
    out = np.empty(9)
    lib().orc_collide_ad(np.ascontiguousarray(pop, dtype=np.float64), X, jx, jy, omega1, ux, uy, out)
    return out


def splitmix64(seed: int, k: int) -> int:
    return int(lib().orc_splitmix64(seed, k))


def grad_periodic(X):
    X = np.ascontiguousarray(X, dtype=np.float64)
    ny, nx = X.shape
    gx = np.empty_like(X)
    gy = np.empty_like(X)
    lib().orc_grad_periodic(X, nx, ny, gx, gy)
    return gx, gy
