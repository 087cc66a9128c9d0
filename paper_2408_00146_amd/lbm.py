"""Thin ctypes binding of ``liblbm_hip.so`` (the C ABI declared in include/lbm.h).

Argument marshalling only: every step of the method runs in the HIP kernels.
PyTorch provides the device workspace and the stream.  There is no CPU
fallback: without the built library or a GPU every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "liblbm_hip.so")

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_NONFINITE, LBM_E_STATE = 0, -1, -2, -3, -4, -5
FP64, FP32, FP16S = 0, 1, 2

FIELD_BITS = {
    "phi": 0, "p": 1, "ux": 2, "uy": 3, "T": 4, "psi": 5,
    "dphi_dx": 6, "dphi_dy": 7, "kappa": 8, "sigma": 9, "Fs_x": 10, "Fs_y": 11, "Fp_x": 12, "Fp_y": 13,
    "R_x": 14, "R_y": 15, "omega_nu": 16, "p_star": 17,
}
MACRO_FIELDS = ("phi", "p", "ux", "uy", "T", "psi")


class LbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"lbm error {code}: {msg}")
        self.code = code


class LbmCase(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("precision", C.c_int32), ("sigma_law", C.c_int32),
        ("init_kind", C.c_int32),
        ("wall", C.c_uint8 * 4), ("t_bc", C.c_uint8 * 4), ("psi_bc", C.c_uint8 * 4), ("reserved0", C.c_uint8 * 4),
        ("psi_w", C.c_double * 4),
        ("T0", C.c_double), ("gradT", C.c_double), ("xT0", C.c_double),
        ("sigma0", C.c_double), ("sigma_T", C.c_double), ("sigma_TT", C.c_double), ("T_ref", C.c_double),
        ("beta_s", C.c_double), ("psi_inf", C.c_double),
        ("rho_A", C.c_double), ("rho_B", C.c_double), ("nu_A", C.c_double), ("nu_B", C.c_double),
        ("alpha_A", C.c_double), ("alpha_B", C.c_double), ("D_psi", C.c_double), ("M_phi", C.c_double),
        ("W", C.c_double), ("s_lam", C.c_double), ("w_lam", C.c_double),
        ("Fext_x", C.c_double), ("Fext_y", C.c_double), ("gravity", C.c_double),
        ("xc", C.c_double), ("yc", C.c_double), ("R", C.c_double),
        ("psi_bulk", C.c_double), ("psi_band", C.c_double), ("psi_gradx", C.c_double), ("phi_noise", C.c_double),
        ("p_jump", C.c_double), ("seed", C.c_uint64), ("max_steps", C.c_int64),
    ]


class LbmDiag(C.Structure):
    _fields_ = [(k, C.c_double) for k in ("mass_phi", "mass_psi", "xc", "yc", "ux", "uy", "p_in", "p_out",
                                          "phi_min", "phi_max", "psi_min", "psi_max", "nonfinite")] + \
               [("step", C.c_int64)]


_ARRAYS = ("wall", "t_bc", "psi_bc", "psi_w")


def make_case(params: dict) -> LbmCase:
    c = LbmCase()
    for name, _ in LbmCase._fields_:
        if name == "reserved0":
            continue
        if name not in params:
            raise KeyError(f"case is missing '{name}'")
        v = params[name]
        if name in _ARRAYS:
            arr = getattr(c, name)
            for k in range(4):
                arr[k] = v[k]
        else:
            setattr(c, name, v)
    return c


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2408_00146_amd.build` "
                               "(or __graft_entry__.build()); there is no CPU fallback")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, u32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_size_t
        L.lbm_last_error.restype = C.c_char_p
        L.lbm_workspace_bytes.restype = sz
        L.lbm_workspace_bytes.argtypes = [C.POINTER(LbmCase), i32]
        L.lbm_init.argtypes = [C.POINTER(LbmCase), i32, vp, sz, vp, C.POINTER(vp)]
        L.lbm_step.argtypes = [vp, i64]
        L.lbm_moments.argtypes = [vp, i32, u32, vp, i32]
        L.lbm_moments_static.argtypes = [vp, i32, u32, vp]
        L.lbm_get_populations.argtypes = [vp, i32, vp, i32]
        L.lbm_set_populations.argtypes = [vp, i32, vp, i32]
        L.lbm_load_fields.argtypes = [vp, i32, vp, vp, vp, i32]
        L.lbm_reduce.argtypes = [vp, i32, C.POINTER(LbmDiag)]
        L.lbm_autotune.argtypes = [vp, i32]
        L.lbm_tile_count.argtypes = []
        L.lbm_tile_shape.argtypes = [i32, C.POINTER(i32), C.POINTER(i32)]
        L.lbm_tile_kind.argtypes = [i32]
        L.lbm_tile_threads.argtypes = [i32]
        L.lbm_set_tile.argtypes = [vp, i32]
        L.lbm_get_tile.argtypes = [vp]
        L.lbm_set_graph.argtypes = [vp, i32]
        L.lbm_steps_done.restype = i64
        L.lbm_steps_done.argtypes = [vp, i32]
        L.lbm_set_kernel_timing.argtypes = [vp, i32]
        L.lbm_kernel_time_ms.argtypes = [vp, C.POINTER(C.c_double), C.POINTER(i64)]
        L.lbm_destroy.argtypes = [vp]
        _lib = L
    return _lib


def _check(rc: int, allow=()):
    if rc != LBM_OK and rc not in allow:
        raise LbmError(rc, lib().lbm_last_error().decode())
    return rc


def tile_shapes() -> list[tuple[int, int]]:
    out = []
    for i in range(lib().lbm_tile_count()):
        bx, by = C.c_int32(), C.c_int32()
        _check(lib().lbm_tile_shape(i, C.byref(bx), C.byref(by)))
        out.append((bx.value, by.value))
    return out


def tile_threads() -> list[int]:
    """Threads per workgroup of every step configuration index."""
    out = []
    for i in range(lib().lbm_tile_count()):
        n = int(lib().lbm_tile_threads(i))
        if n <= 0:
            _check(n)
        out.append(n)
    return out


def config_name(index: int) -> str:
    """'tile BXxBY/threads' of a step configuration index."""
    bx, by = tile_shapes()[index]
    return f"{tile_kinds()[index]} {bx}x{by}/{tile_threads()[index]}"


KINDS = {0: "tile"}


def tile_kinds() -> list[str]:
    """Kind of every step configuration index: 'tile' (one workgroup per
    tile), 'walk' (resident workgroups walking the tile table) or 'walkpf'
    (the walk with next-tile prefetch)."""
    return [KINDS[lib().lbm_tile_kind(i)] for i in range(lib().lbm_tile_count())]


def workspace_bytes(cases: list[dict]) -> int:
    arr = (LbmCase * len(cases))(*[make_case(c) for c in cases])
    return int(lib().lbm_workspace_bytes(arr, len(cases)))


class Solver:
    """A set of cases advanced together on one GPU."""

    def __init__(self, cases, device: str = "cuda:0", stream=None):
        import torch

        if isinstance(cases, dict):
            cases = [cases]
        self.cases = [dict(c) for c in cases]
        self.device = torch.device(device)
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the lattice Boltzmann step runs only on the GPU")
        self._torch = torch
        # A stream of its own (default priority): the legacy NULL stream cannot
        # be captured into a hipGraph.  Every tensor the solver touches is
        # allocated and filled under this stream, so all work stays ordered.
        self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
        arr = (LbmCase * len(self.cases))(*[make_case(c) for c in self.cases])
        self._arr = arr
        nbytes = int(lib().lbm_workspace_bytes(arr, len(self.cases)))
        h = C.c_void_p()
        with torch.cuda.device(self.device), torch.cuda.stream(self.stream):
            self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
            base = self.workspace.data_ptr()
            self._ws_ptr = (base + 255) & ~255
            _check(lib().lbm_init(arr, len(self.cases), C.c_void_p(self._ws_ptr), nbytes,
                                  C.c_void_p(self.stream.cuda_stream), C.byref(h)))
        self._h = h

    def _on_stream(self):
        return self._torch.cuda.stream(self.stream)

    # -------------------------------------------------------------- lifecycle
    def close(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            lib().lbm_destroy(h)
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

    # ------------------------------------------------------------------- step
    def step(self, n: int = 1):
        _check(lib().lbm_step(self._h, int(n)))
        return self

    def steps_done(self, case: int = 0) -> int:
        return int(lib().lbm_steps_done(self._h, case))

    def synchronize(self):
        self.stream.synchronize()

    # ------------------------------------------------------------ inspection
    def fields(self, case: int = 0, names=MACRO_FIELDS, device: bool = False) -> dict:
        torch = self._torch
        mask = 0
        for k in names:
            mask |= 1 << FIELD_BITS[k]
        ordered = sorted(names, key=lambda k: FIELD_BITS[k])
        nx, ny = self.cases[case]["nx"], self.cases[case]["ny"]
        with self._on_stream():
            out = torch.empty((len(ordered), ny, nx), dtype=torch.float64, device=self.device)
            _check(lib().lbm_moments(self._h, case, mask, C.c_void_p(out.data_ptr()), 1))
            if not device:
                out = out.cpu().numpy()
        return {k: out[i] for i, k in enumerate(ordered)}

    def fields_static(self, case: int = 0, names=MACRO_FIELDS) -> dict:
        """The fields of `fields`, fetched through lbm_moments_static (host
        destination, staged through the library's fixed device array: no
        device allocation)."""
        mask = 0
        for k in names:
            mask |= 1 << FIELD_BITS[k]
        ordered = sorted(names, key=lambda k: FIELD_BITS[k])
        nx, ny = self.cases[case]["nx"], self.cases[case]["ny"]
        out = np.empty((len(ordered), ny, nx), dtype=np.float64)
        _check(lib().lbm_moments_static(self._h, case, mask, out.ctypes.data_as(C.c_void_p)))
        return {k: out[i] for i, k in enumerate(ordered)}

    def populations(self, case: int = 0) -> np.ndarray:
        torch = self._torch
        nx, ny = self.cases[case]["nx"], self.cases[case]["ny"]
        with self._on_stream():
            out = torch.empty((4, 9, ny, nx), dtype=torch.float64, device=self.device)
            _check(lib().lbm_get_populations(self._h, case, C.c_void_p(out.data_ptr()), 1))
            return out.cpu().numpy()

    def set_populations(self, pops, case: int = 0):
        torch = self._torch
        with self._on_stream():
            t = torch.as_tensor(np.ascontiguousarray(pops, dtype=np.float64)).to(self.device)
            _check(lib().lbm_set_populations(self._h, case, C.c_void_p(t.data_ptr()), 1))
        self.synchronize()

    def load_fields(self, phi, T, psi, case: int = 0):
        torch = self._torch
        nx, ny = self.cases[case]["nx"], self.cases[case]["ny"]
        with self._on_stream():
            ts = [torch.from_numpy(np.broadcast_to(np.asarray(v, dtype=np.float64), (ny, nx)).copy()).to(self.device)
                  for v in (phi, T, psi)]
            _check(lib().lbm_load_fields(self._h, case, *[C.c_void_p(t.data_ptr()) for t in ts], 1))
        self.synchronize()

    def reduce(self, case: int = 0, allow_nonfinite: bool = False) -> dict:
        d = LbmDiag()
        _check(lib().lbm_reduce(self._h, case, C.byref(d)), allow=(LBM_E_NONFINITE,) if allow_nonfinite else ())
        return {k: getattr(d, k) for k, _ in LbmDiag._fields_}

    # ----------------------------------------------------------------- tuning
    def autotune(self, trial_steps: int = 20) -> int:
        _check(lib().lbm_autotune(self._h, int(trial_steps)))
        return self.tile

    @property
    def tile(self) -> int:
        return int(lib().lbm_get_tile(self._h))

    def set_tile(self, index: int):
        _check(lib().lbm_set_tile(self._h, int(index)))

    def set_graph(self, enable: bool):
        _check(lib().lbm_set_graph(self._h, 1 if enable else 0))

    def set_kernel_timing(self, mode):
        """0/False off, 1/True: each step launched alone between events,
        2: events around each launched chunk (graph replay)."""
        _check(lib().lbm_set_kernel_timing(self._h, int(mode)))

    def kernel_time_ms(self) -> tuple[float, int]:
        ms, n = C.c_double(), C.c_int64()
        _check(lib().lbm_kernel_time_ms(self._h, C.byref(ms), C.byref(n)))
        return ms.value, n.value
