"""ctypes binding of libasd (include/asd.h).

Argument marshalling only: every step of the sLLG path runs in the HIP
kernels of libasd.so.  PyTorch supplies device memory (one uint8 workspace
tensor per handle) and the HIP stream.  Importing this module does not touch
the GPU; loading the library fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libasd.so")

ASD_OK, ASD_EINVAL, ASD_ENOMEM, ASD_EHIP, ASD_ESTATE, ASD_ENONFINITE, ASD_EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6)
ASD_FP64, ASD_FP32 = 0, 1
ASD_SC, ASD_L10 = 0, 1
ASD_BC_OPEN, ASD_BC_PERIODIC, ASD_BC_TRACK = 0, 1, 2
ASD_SPOT_NONE, ASD_SPOT_MOVING, ASD_SPOT_LOCKED = 0, 1, 2
ASD_KERNEL_AUTO, ASD_KERNEL_PLAIN, ASD_KERNEL_FUSED = 0, 1, 2
ASD_CONE_PRINTED, ASD_CONE_CAP = 0, 1
ASD_DEMAG_EACH_STAGE, ASD_DEMAG_ONCE = 0, 1

SYMBOLS = [
    "asd_workspace_bytes", "asd_create", "asd_destroy", "asd_set_field_temperature",
    "asd_set_spins", "asd_get_spins", "asd_step", "asd_prepare", "asd_shift_window",
    "asd_reduce_magnetization", "asd_reduce_magnetization_static", "asd_reduce_energy", "asd_accumulate_moments",
    "asd_get_moment_stats", "asd_grain_count", "asd_stored_sites", "asd_get_grain_labels",
    "asd_neighbour_count", "asd_get_neighbours", "asd_host_grain_labels", "asd_host_neighbours",
    "asd_coarse_grain", "asd_thermalise_columns", "asd_demag_field", "asd_mc_sweep",
    "asd_get_state", "asd_set_step", "asd_philox",
    "asd_autotune", "asd_set_variant", "asd_get_variant", "asd_variant_count", "asd_variant_name",
    "asd_strerror",
    "asd_last_error",
    "asd_mm_workspace_bytes", "asd_mm_create", "asd_mm_destroy", "asd_mm_set_field_temperature",
    "asd_mm_set_m", "asd_mm_get_m", "asd_mm_step", "asd_mm_get_step", "asd_mm_last_error",
    "asd_mm_set_face", "asd_mm_get_face", "asd_multiscale_step", "asd_multiscale_shift",
    "asd_set_cone_reading", "asd_set_demag_reading", "asd_set_columns", "asd_msd_workspace_bytes", "asd_msd_create",
    "asd_msd_destroy", "asd_multiscale_step_demag", "asd_msd_fields",
    "asd_window_size", "asd_get_stream",
]


class AsdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libasd error {code}: {msg}")
        self.code = code


class asd_params(C.Structure):
    _fields_ = [("lattice", C.c_int32), ("precision", C.c_int32), ("a", C.c_double),
                ("c", C.c_double), ("n_shells", C.c_int32), ("J", C.c_double * 4),
                ("mu_s", C.c_double), ("alpha", C.c_double), ("gamma", C.c_double),
                ("dt", C.c_double), ("k_u", C.c_double), ("seed", C.c_uint64),
                ("philox_rounds", C.c_int32), ("kernel", C.c_int32), ("graph_steps", C.c_int32),
                ("demag_cell", C.c_int32 * 3)]


class asd_mm_params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("bc_x", C.c_int32), ("bc_y", C.c_int32), ("bc_z", C.c_int32),
                ("h", C.c_double * 3), ("Ms0", C.c_double), ("A0", C.c_double),
                ("K0", C.c_double), ("lambda_", C.c_double), ("gamma", C.c_double),
                ("Tc", C.c_double), ("mu_s", C.c_double), ("dt", C.c_double),
                ("graph_steps", C.c_int32)]


class asd_system_desc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("bc_x", C.c_int32),
                ("bc_y", C.c_int32), ("bc_z", C.c_int32), ("track_nx", C.c_int32),
                ("n_seeds", C.c_int32), ("seeds_xy", C.POINTER(C.c_int32)),
                ("voronoi_q", C.c_int32), ("boundary_w_units", C.c_int64),
                ("labels", C.POINTER(C.c_int32)), ("k_u_grain", C.POINTER(C.c_double)),
                ("n_k_u_grain", C.c_int32), ("T_system", C.c_double)]


class asd_drive(C.Structure):
    _fields_ = [("B", C.c_double * 3), ("n_bits", C.c_int32), ("bits", C.POINTER(C.c_uint8)),
                ("steps_per_bit", C.c_int64), ("spot_mode", C.c_int32), ("T_amb", C.c_double),
                ("T_peak", C.c_double), ("fwhm", C.c_double), ("x0", C.c_double),
                ("y0", C.c_double), ("v", C.c_double)]


_lib = None


def lib():
    """Load libasd.so (built in-tree); raise if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built: run paper_2502_02236_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P = C.POINTER
        vp = C.c_void_p
        h = vp
        L.asd_workspace_bytes.argtypes = [P(asd_params), P(asd_system_desc), C.c_int32, P(C.c_size_t)]
        L.asd_create.argtypes = [P(asd_params), P(asd_system_desc), C.c_int32, vp, C.c_size_t, vp, P(vp)]
        L.asd_destroy.argtypes = [h]
        L.asd_set_field_temperature.argtypes = [h, P(asd_drive)]
        L.asd_set_spins.argtypes = [h, C.c_int32, vp, C.c_int32]
        L.asd_get_spins.argtypes = [h, C.c_int32, vp, C.c_int32]
        L.asd_step.argtypes = [h, C.c_int64]
        L.asd_prepare.argtypes = [h]
        L.asd_shift_window.argtypes = [h, C.c_int32]
        L.asd_reduce_magnetization.argtypes = [h, vp, vp]
        L.asd_reduce_magnetization_static.argtypes = [h, vp, vp]
        L.asd_reduce_energy.argtypes = [h, vp]
        L.asd_accumulate_moments.argtypes = [h, C.c_int32]
        L.asd_get_moment_stats.argtypes = [h, vp]
        L.asd_grain_count.argtypes = [h, C.c_int32, P(C.c_int32)]
        L.asd_stored_sites.argtypes = [h, C.c_int32, P(C.c_int64)]
        L.asd_get_grain_labels.argtypes = [h, C.c_int32, vp]
        L.asd_neighbour_count.argtypes = [h, C.c_int32, P(C.c_int64)]
        L.asd_get_neighbours.argtypes = [h, C.c_int32, vp, vp, vp]
        L.asd_host_grain_labels.argtypes = [P(asd_params), P(asd_system_desc), vp]
        L.asd_host_neighbours.argtypes = [P(asd_params), P(asd_system_desc), P(C.c_int64), vp, vp, vp]
        L.asd_get_state.argtypes = [h, C.c_int32, P(C.c_int64), P(C.c_int32)]
        L.asd_set_step.argtypes = [h, C.c_int64]
        L.asd_philox.argtypes = [C.c_uint64, C.c_int32, vp, vp, C.c_int64, vp]
        L.asd_autotune.argtypes = [h, C.c_char_p]
        L.asd_set_variant.argtypes = [h, C.c_int32, C.c_int32]
        L.asd_get_variant.argtypes = [h, P(C.c_int32), P(C.c_int32)]
        L.asd_coarse_grain.argtypes = [h, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                       C.c_int32, vp]
        L.asd_thermalise_columns.argtypes = [h, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                             C.c_int32, C.c_int32, vp, C.c_uint32]
        L.asd_demag_field.argtypes = [h, vp, vp]
        L.asd_mc_sweep.argtypes = [h, C.c_int64]
        L.asd_variant_count.argtypes = [h, C.c_int32, P(C.c_int32)]
        L.asd_mm_workspace_bytes.argtypes = [P(asd_mm_params), P(C.c_size_t)]
        L.asd_mm_create.argtypes = [P(asd_mm_params), vp, C.c_size_t, vp, P(vp)]
        L.asd_mm_destroy.argtypes = [vp]
        L.asd_mm_set_field_temperature.argtypes = [vp, P(asd_drive)]
        L.asd_mm_set_m.argtypes = [vp, vp, C.c_int32]
        L.asd_mm_get_m.argtypes = [vp, vp, C.c_int32]
        L.asd_mm_step.argtypes = [vp, C.c_int64]
        L.asd_mm_get_step.argtypes = [vp, P(C.c_int64)]
        L.asd_mm_set_face.argtypes = [vp, C.c_int32, vp, C.c_int32]
        L.asd_mm_get_face.argtypes = [vp, C.c_int32, vp]
        L.asd_multiscale_step.argtypes = [h, C.c_int32, vp, vp, C.c_int32, C.c_int32, C.c_int32,
                                          C.c_int64]
        L.asd_multiscale_shift.argtypes = [h, C.c_int32, vp, vp, C.c_int32, C.c_int32, C.c_int32,
                                           vp, vp]
        L.asd_set_cone_reading.argtypes = [h, C.c_int32]
        L.asd_set_demag_reading.argtypes = [h, C.c_int32]
        L.asd_msd_workspace_bytes.argtypes = [h, C.c_int32, vp, vp, C.c_int32, C.c_int32, C.c_int32,
                                              P(C.c_size_t)]
        L.asd_msd_create.argtypes = [h, C.c_int32, vp, vp, C.c_int32, C.c_int32, C.c_int32, vp,
                                     C.c_size_t, P(vp)]
        L.asd_msd_destroy.argtypes = [vp]
        L.asd_multiscale_step_demag.argtypes = [vp, C.c_int64]
        L.asd_msd_fields.argtypes = [vp, vp, vp, vp]
        L.asd_set_columns.argtypes = [h, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                      C.c_int32, vp]
        L.asd_window_size.argtypes = [h, C.c_int32, P(C.c_int32), P(C.c_int32), P(C.c_int32)]
        L.asd_get_stream.argtypes = [h, P(vp)]
        L.asd_mm_last_error.argtypes = [vp]
        L.asd_mm_last_error.restype = C.c_char_p
        L.asd_variant_name.argtypes = [h, C.c_char_p, C.c_size_t]
        L.asd_strerror.argtypes = [C.c_int]
        L.asd_strerror.restype = C.c_char_p
        L.asd_last_error.argtypes = [h]
        L.asd_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _check(rc, handle=None):
    if rc != ASD_OK:
        msg = lib().asd_last_error(handle).decode(errors="replace")
        raise AsdError(rc, f"{lib().asd_strerror(rc).decode()}: {msg}")
    return rc


def _np_ptr(a, ctype=None):
    return None if a is None else a.ctypes.data_as(C.c_void_p if ctype is None else C.POINTER(ctype))


# ----------------------------------------------------------------- same-named wrappers
def asd_workspace_bytes(params, systems):
    arr = (asd_system_desc * len(systems))(*systems)
    out = C.c_size_t(0)
    _check(lib().asd_workspace_bytes(C.byref(params), arr, len(systems), C.byref(out)))
    return out.value


def asd_create(params, systems, workspace_ptr, workspace_bytes, stream_ptr):
    arr = (asd_system_desc * len(systems))(*systems)
    h = C.c_void_p()
    _check(lib().asd_create(C.byref(params), arr, len(systems), C.c_void_p(workspace_ptr),
                            workspace_bytes, C.c_void_p(stream_ptr), C.byref(h)))
    return h


def asd_destroy(h):
    _check(lib().asd_destroy(h))


def asd_set_field_temperature(h, drive):
    _check(lib().asd_set_field_temperature(h, C.byref(drive)), h)


def asd_set_spins(h, sys, ptr, on_device):
    _check(lib().asd_set_spins(h, sys, C.c_void_p(ptr), int(on_device)), h)


def asd_get_spins(h, sys, ptr, on_device):
    _check(lib().asd_get_spins(h, sys, C.c_void_p(ptr), int(on_device)), h)


def asd_step(h, n):
    _check(lib().asd_step(h, int(n)), h)


def asd_prepare(h):
    """Capture the step graphs now (no work is enqueued)."""
    _check(lib().asd_prepare(h), h)


def asd_shift_window(h, columns):
    _check(lib().asd_shift_window(h, int(columns)), h)


def asd_reduce_magnetization(h, per_grain, per_system):
    return lib().asd_reduce_magnetization(h, _np_ptr(per_grain), _np_ptr(per_system))


def asd_reduce_magnetization_static(h, per_grain, per_system):
    return lib().asd_reduce_magnetization_static(h, _np_ptr(per_grain), _np_ptr(per_system))


def asd_reduce_energy(h, per_system):
    return lib().asd_reduce_energy(h, _np_ptr(per_system))


def asd_accumulate_moments(h, reset):
    _check(lib().asd_accumulate_moments(h, int(reset)), h)


def asd_get_moment_stats(h, out):
    return lib().asd_get_moment_stats(h, _np_ptr(out))


def asd_philox(seed, rounds, ctr_ptr, out_ptr, n, stream_ptr):
    _check(lib().asd_philox(seed, rounds, C.c_void_p(ctr_ptr), C.c_void_p(out_ptr), n,
                            C.c_void_p(stream_ptr)))


def asd_host_grain_labels(params, system, n_stored):
    """Grain labels built on the host (no device)."""
    out = np.empty(n_stored, dtype=np.int32)
    rc = lib().asd_host_grain_labels(C.byref(params), C.byref(system), _np_ptr(out))
    if rc not in (ASD_OK, ASD_EUNSUPPORTED):
        _check(rc)
    return out


def asd_host_neighbours(params, system):
    """CSR neighbour table built on the host (no device)."""
    n = C.c_int64()
    _check(lib().asd_host_neighbours(C.byref(params), C.byref(system), C.byref(n), None, None, None))
    per = 1 if params.lattice == ASD_SC else 2
    sx = system.track_nx if system.bc_x == ASD_BC_TRACK else system.nx
    ns = per * sx * system.ny * system.nz
    row = np.empty(ns + 1, dtype=np.int64)
    col = np.empty(max(n.value, 1), dtype=np.int32)
    sh = np.empty(max(n.value, 1), dtype=np.int8)
    _check(lib().asd_host_neighbours(C.byref(params), C.byref(system), C.byref(n), _np_ptr(row),
                                     _np_ptr(col), _np_ptr(sh)))
    return row, col[:n.value], sh[:n.value]


def asd_set_variant(h, kernel, tile):
    _check(lib().asd_set_variant(h, kernel, tile), h)


def asd_get_variant(h):
    k, t = C.c_int32(), C.c_int32()
    _check(lib().asd_get_variant(h, C.byref(k), C.byref(t)), h)
    return k.value, t.value


def asd_autotune(h, cache_path=None):
    _check(lib().asd_autotune(h, None if cache_path is None else cache_path.encode()), h)


# ----------------------------------------------------------------- convenience wrapper
class Handle:
    """One libasd handle with its torch-owned workspace and a dedicated stream."""

    def __init__(self, params: asd_params, systems: list, device: str = "cuda:0", stream=None):
        import torch  # device memory and streams only

        self.torch = torch
        self.device = torch.device(device)
        self._keep = []  # host arrays referenced by descriptors during create
        self.params = params
        self.systems = systems
        nbytes = asd_workspace_bytes(params, systems)
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self.ws_ptr = (base + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.h = asd_create(params, systems, self.ws_ptr, nbytes, self.stream.cuda_stream)
        self.dtype = np.float64 if params.precision == ASD_FP64 else np.float32

    def close(self):
        if getattr(self, "h", None):
            asd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- drive and state
    def set_drive(self, drive: asd_drive):
        asd_set_field_temperature(self.h, drive)

    def stored_sites(self, sys: int = 0) -> int:
        n = C.c_int64()
        _check(lib().asd_stored_sites(self.h, sys, C.byref(n)), self.h)
        return n.value

    def grain_count(self, sys: int = 0) -> int:
        n = C.c_int32()
        _check(lib().asd_grain_count(self.h, sys, C.byref(n)), self.h)
        return n.value

    def set_spins(self, S, sys: int = 0):
        """S: [3, n_stored] host array (converted to the handle precision) or device tensor."""
        if hasattr(S, "data_ptr"):
            asd_set_spins(self.h, sys, S.data_ptr(), True)
        else:
            a = np.ascontiguousarray(S, dtype=self.dtype).reshape(3, -1)
            if a.shape[1] != self.stored_sites(sys):
                raise ValueError("spin array does not match the stored lattice")
            asd_set_spins(self.h, sys, a.ctypes.data, False)

    def get_spins(self, sys: int = 0) -> np.ndarray:
        out = np.empty((3, self.stored_sites(sys)), dtype=self.dtype)
        asd_get_spins(self.h, sys, out.ctypes.data, False)
        return out

    def step(self, n: int):
        asd_step(self.h, n)

    def prepare(self):
        asd_prepare(self.h)

    def coarse_cells(self, sys: int, ncols: int, cx: int, cy: int, cz: int) -> int:
        d = self.systems[sys]
        return -(-ncols // cx) * -(-d.ny // cy) * -(-d.nz // cz)

    def coarse_grain(self, sys: int, x0: int, ncols: int, cx: int, cy: int, cz: int, out=None):
        """Eq. 6 sums per coarse cell: [ncell, 4] (sum m, N), float64 device tensor
        (complete when this returns)."""
        torch = self.torch
        n = self.coarse_cells(sys, ncols, cx, cy, cz)
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float64, device=self.device)
        _check(lib().asd_coarse_grain(self.h, sys, x0, ncols, cx, cy, cz, out.data_ptr()), self.h)
        self.stream.synchronize()
        return out

    def thermalise_columns(self, sys: int, x0: int, ncols: int, cx: int, cy: int, cz: int, mcell,
                           step: int):
        """Cone spins around the reduced magnetisation mcell [ncell, 3] (host array or
        device tensor) of each coarse cell (complete when this returns)."""
        torch = self.torch
        m = torch.as_tensor(mcell, dtype=torch.float64, device=self.device).contiguous()
        if m.numel() != 3 * self.coarse_cells(sys, ncols, cx, cy, cz):
            raise ValueError("mcell must hold 3 values per coarse cell")
        torch.cuda.current_stream(self.device).synchronize()  # the upload is complete
        _check(lib().asd_thermalise_columns(self.h, sys, x0, ncols, cx, cy, cz, m.data_ptr(),
                                            step), self.h)
        self.stream.synchronize()

    def set_cone_reading(self, reading: int):
        """ASD_CONE_PRINTED (default) or ASD_CONE_CAP for the inverse transfer."""
        _check(lib().asd_set_cone_reading(self.h, reading), self.h)

    def set_demag_reading(self, reading: int):
        """ASD_DEMAG_EACH_STAGE (default): the demagnetising field at both Heun
        stages; ASD_DEMAG_ONCE: once per step, held through both stages."""
        _check(lib().asd_set_demag_reading(self.h, reading), self.h)

    def mc_sweep(self, n: int):
        """n Metropolis sweeps at each system's ambient temperature."""
        _check(lib().asd_mc_sweep(self.h, n), self.h)

    def demag_field(self):
        """Demagnetising flux density mu0 H_d (T) of the current spins per coarse
        cell: float64 [n_sys, 3, ncell], and the mesh (ncx, ncy, ncz)."""
        p = self.params
        cx, cy, cz = (int(v) for v in p.demag_cell)
        d = self.systems[0]
        ncell = -(-d.nx // cx) * -(-d.ny // cy) * -(-d.nz // cz) if cx else 0
        out = np.zeros((len(self.systems), 3, max(ncell, 1)))
        mesh = np.zeros(3, dtype=np.int32)
        _check(lib().asd_demag_field(self.h, out.ctypes.data, mesh.ctypes.data), self.h)
        return out[:, :, :ncell], tuple(int(v) for v in mesh)

    def shift_window(self, columns: int):
        asd_shift_window(self.h, columns)

    def synchronize(self):
        self.stream.synchronize()

    def magnetization(self):
        ng = sum(self.grain_count(s) for s in range(len(self.systems)))
        pg = np.zeros((max(ng, 1), 4))
        ps = np.zeros((len(self.systems), 4))
        _check(asd_reduce_magnetization(self.h, pg, ps), self.h)
        return pg[:ng], ps

    def energy(self):
        out = np.zeros((len(self.systems), 4))
        _check(asd_reduce_energy(self.h, out), self.h)
        return out

    def accumulate_moments(self, reset=False):
        asd_accumulate_moments(self.h, reset)

    def moment_stats(self):
        out = np.zeros((len(self.systems), 5))
        _check(asd_get_moment_stats(self.h, out), self.h)
        return out

    def labels(self, sys: int = 0) -> np.ndarray:
        out = np.empty(self.stored_sites(sys), dtype=np.int32)
        _check(lib().asd_get_grain_labels(self.h, sys, _np_ptr(out)), self.h)
        return out

    def neighbours(self, sys: int = 0):
        n = C.c_int64()
        _check(lib().asd_neighbour_count(self.h, sys, C.byref(n)), self.h)
        ns = self.stored_sites(sys)
        row = np.empty(ns + 1, dtype=np.int64)
        col = np.empty(max(n.value, 1), dtype=np.int32)
        sh = np.empty(max(n.value, 1), dtype=np.int8)
        _check(lib().asd_get_neighbours(self.h, sys, _np_ptr(row), _np_ptr(col), _np_ptr(sh)), self.h)
        return row, col[:n.value], sh[:n.value]

    def state(self, sys: int = 0):
        st, org = C.c_int64(), C.c_int32()
        _check(lib().asd_get_state(self.h, sys, C.byref(st), C.byref(org)), self.h)
        return st.value, org.value

    def set_step(self, step: int):
        _check(lib().asd_set_step(self.h, step), self.h)

    def set_variant(self, kernel: int, tile: int = 0):
        asd_set_variant(self.h, kernel, tile)

    def variant(self):
        return asd_get_variant(self.h)

    def variant_count(self, kernel: int) -> int:
        """Number of tile variants of a kernel family."""
        n = C.c_int32()
        _check(lib().asd_variant_count(self.h, kernel, C.byref(n)), self.h)
        return n.value

    def variant_name(self) -> str:
        buf = C.create_string_buffer(256)
        _check(lib().asd_variant_name(self.h, buf, 256), self.h)
        return buf.value.decode()

    def autotune(self, cache_path=None):
        asd_autotune(self.h, cache_path)


# ----------------------------------------------------------------- micromagnetic region
def _mm_check(rc, handle=None):
    if rc != ASD_OK:
        msg = lib().asd_mm_last_error(handle).decode(errors="replace")
        raise AsdError(rc, f"{lib().asd_strerror(rc).decode()}: {msg}")
    return rc


class MMHandle:
    """A micromagnetic region (asd_mm_*) with a torch-owned workspace and its own stream."""

    def __init__(self, params: asd_mm_params, device: str = "cuda:0", stream=None):
        """stream: a torch stream to share (a multiscale window runs both kinds of
        handle on the atomistic handle's stream)."""
        import torch

        self.torch = torch
        self.device = torch.device(device)
        self.params = params
        nb = C.c_size_t()
        _mm_check(lib().asd_mm_workspace_bytes(C.byref(params), C.byref(nb)))
        self.workspace = torch.empty(nb.value + 256, dtype=torch.uint8, device=self.device)
        ptr = (self.workspace.data_ptr() + 255) // 256 * 256
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        out = C.c_void_p()
        _mm_check(lib().asd_mm_create(C.byref(params), ptr, nb.value, self.stream.cuda_stream,
                                      C.byref(out)))
        self.h = out.value
        self.n = params.nx * params.ny * params.nz
        self.dtype = np.float64 if params.precision == ASD_FP64 else np.float32

    def close(self):
        if getattr(self, "h", None):
            lib().asd_mm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_drive(self, drive: asd_drive):
        _mm_check(lib().asd_mm_set_field_temperature(self.h, C.byref(drive)), self.h)

    def set_m(self, m):
        a = np.ascontiguousarray(m, dtype=self.dtype).reshape(3, -1)
        if a.shape[1] != self.n:
            raise ValueError("magnetisation array does not match the mesh")
        _mm_check(lib().asd_mm_set_m(self.h, a.ctypes.data, 0), self.h)

    def get_m(self) -> np.ndarray:
        out = np.empty((3, self.n), dtype=self.dtype)
        _mm_check(lib().asd_mm_get_m(self.h, out.ctypes.data, 0), self.h)
        return out

    def step(self, n: int):
        _mm_check(lib().asd_mm_step(self.h, n), self.h)

    def step_count(self) -> int:
        v = C.c_int64()
        _mm_check(lib().asd_mm_get_step(self.h, C.byref(v)), self.h)
        return v.value


def multiscale_step(atoms: "Handle", sys: int, left, right, cell, n: int):
    """n coupled steps of micromagnetic regions left/right (MMHandle or None) and the
    atomistic window of track system `sys` (all on atoms.stream)."""
    rc = lib().asd_multiscale_step(atoms.h, sys, left.h if left else None,
                                   right.h if right else None, cell[0], cell[1], cell[2], n)
    if rc != ASD_OK:
        raise AsdError(rc, lib().asd_strerror(rc).decode())


def multiscale_shift(atoms: "Handle", sys: int, left, right, cell, enter=None, leave=None):
    """Move the multiscale window by one coarse cell along +x (asd_multiscale_shift).
    enter: the right region's new last column [ny*nz, 3] (host array or device
    tensor); leave: optional float64 device tensor [ny*nz, 3] for the left region's
    leaving column.  Complete when this returns."""
    torch = atoms.torch
    ent = None
    if enter is not None:
        ent = torch.as_tensor(enter, dtype=torch.float64, device=atoms.device).contiguous()
        torch.cuda.current_stream(atoms.device).synchronize()  # the upload is complete
    rc = lib().asd_multiscale_shift(atoms.h, sys, left.h if left else None,
                                    right.h if right else None, cell[0], cell[1], cell[2],
                                    ent.data_ptr() if ent is not None else None,
                                    leave.data_ptr() if leave is not None else None)
    if rc != ASD_OK:
        raise AsdError(rc, lib().asd_strerror(rc).decode())
    atoms.stream.synchronize()


class MultiscaleDemag:
    """The demagnetising field of a whole multiscale window (asd_msd_*): the
    left region, the atomistic window and the right region as one mesh, with
    a torch-owned workspace on the atomistic handle's device."""

    def __init__(self, atoms: "Handle", sys: int, left, right, cell):
        torch = atoms.torch
        self.atoms = atoms
        lh = left.h if left else None
        rh = right.h if right else None
        n = C.c_size_t(0)
        rc = lib().asd_msd_workspace_bytes(atoms.h, sys, lh, rh, cell[0], cell[1], cell[2],
                                           C.byref(n))
        if rc != ASD_OK:
            raise AsdError(rc, lib().asd_mm_last_error(None).decode())
        self.workspace = torch.empty(n.value + 256, dtype=torch.uint8, device=atoms.device)
        base = (self.workspace.data_ptr() + 255) // 256 * 256
        out = C.c_void_p()
        rc = lib().asd_msd_create(atoms.h, sys, lh, rh, cell[0], cell[1], cell[2], base, n.value,
                                  C.byref(out))
        if rc != ASD_OK:
            raise AsdError(rc, lib().asd_mm_last_error(None).decode())
        self.h = out

    def step(self, n: int):
        """n coupled steps with the demagnetising field of the whole window."""
        rc = lib().asd_multiscale_step_demag(self.h, n)
        if rc != ASD_OK:
            raise AsdError(rc, lib().asd_strerror(rc).decode())
        self.atoms.stream.synchronize()

    def fields(self):
        """(all, regions, mesh): the last fields [3, NX ny nz] and (NX, ny, nz)."""
        mesh = np.zeros(3, dtype=np.int32)
        _check_mm(lib().asd_msd_fields(self.h, None, None, _np_ptr(mesh)))
        n = int(np.prod(mesh))
        a = np.zeros((3, n))
        r = np.zeros((3, n))
        _check_mm(lib().asd_msd_fields(self.h, _np_ptr(a), _np_ptr(r), None))
        return a, r, tuple(int(v) for v in mesh)

    def close(self):
        if getattr(self, "h", None):
            lib().asd_msd_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_mm(rc):
    if rc != ASD_OK:
        raise AsdError(rc, lib().asd_mm_last_error(None).decode())
    return rc
