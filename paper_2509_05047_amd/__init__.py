"""Python binding of libsse.so, the MI355X scatter-estimation library.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  Device buffers are torch tensors on the context's GPU (PyTorch
supplies device memory and streams); the C ABI itself takes plain pointers
(see include/sse.h).  Importing this module never falls back to any other
implementation: if libsse.so is missing it raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsse.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, EBUSY = range(6)
F32, F16, BF16 = 0, 1, 2
MEM_HOST, MEM_DEVICE = 0, 1
STAT_NAMES = ["histories", "steps", "real", "compton", "rayleigh", "absorbed", "killed", "capped",
              "escaped", "detected", "in_window", "scatter", "true", "rej_window", "rej_same",
              "rej_ring", "rej_radial", "rej_tof", "rng_blocks", "rej_gap", "gap_assigned"]
STAT_COUNT = len(STAT_NAMES)
RECORD_WORDS = 32
GAP_DISCARD, GAP_NEAREST, GAP_EDGE_LUT = 0, 1, 2
GAP_POLICIES = {"discard": GAP_DISCARD, "nearest": GAP_NEAREST, "edge_lut": GAP_EDGE_LUT}


class SseError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"sse status {status}: {msg}")
        self.status = status


class ScannerDesc(C.Structure):
    _fields_ = [("n_crystals", C.c_int32), ("n_rings", C.c_int32), ("radius_mm", C.c_float),
                ("length_mm", C.c_float), ("crystals_per_module", C.c_int32),
                ("rings_per_block", C.c_int32), ("max_ring_diff", C.c_int32)]


class SinoDesc(C.Structure):
    _fields_ = [("n_rad", C.c_int32), ("n_view", C.c_int32), ("n_plane", C.c_int32), ("n_tof", C.c_int32),
                ("tof_bin_mm", C.c_float), ("tof_sigma_mm", C.c_float)]


class PhysicsDesc(C.Structure):
    _fields_ = [("e_lo_kev", C.c_float), ("e_hi_kev", C.c_float), ("e_kill_kev", C.c_float),
                ("e_fwhm_frac", C.c_float), ("f_compton", C.c_float), ("f_rayleigh", C.c_float),
                ("f_photo", C.c_float), ("rayleigh_beta", C.c_float), ("mu_majorant", C.c_float),
                ("max_interactions", C.c_int32)]


class PhantomDesc(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("voxel_mm", C.c_float * 3), ("lo_mm", C.c_float * 3)]


class LutDesc(C.Structure):
    _fields_ = [("dims", C.c_int32 * 5), ("e_min_kev", C.c_float), ("e_max_kev", C.c_float)]


class GapDesc(C.Structure):
    _fields_ = [("transaxial_gap_rad", C.c_float), ("axial_gap_mm", C.c_float), ("policy", C.c_int32),
                ("edge_n_angle", C.c_int32), ("edge_n_pos", C.c_int32), ("reserved", C.c_int32)]


class EdgeGeom(C.Structure):
    _fields_ = [("gap_mm", C.c_float), ("depth_mm", C.c_float), ("doi_mm", C.c_float),
                ("mu_per_mm", C.c_float), ("n_angle", C.c_int32), ("n_pos", C.c_int32)]


class Outputs(C.Structure):
    _fields_ = [("scatter_counts", C.c_void_p), ("scatter_weights", C.c_void_p),
                ("true_counts", C.c_void_p), ("true_weights", C.c_void_p),
                ("stats", C.c_void_p), ("records", C.c_void_p), ("record_stride", C.c_uint64)]


class ServerCfg(C.Structure):
    _fields_ = [("max_active", C.c_int32), ("reserved", C.c_int32), ("hbm_budget_bytes", C.c_uint64),
                ("tick_histories", C.c_uint64), ("chunk_histories", C.c_uint64)]


class Request(C.Structure):
    _fields_ = [("phantom", C.c_uint32), ("reserved", C.c_uint32), ("n_histories", C.c_uint64),
                ("seed", C.c_uint64), ("h_offset", C.c_uint64), ("scatter_counts", C.c_void_p),
                ("scatter_weights", C.c_void_p)]


class Completion(C.Structure):
    _fields_ = [("id", C.c_uint64), ("status", C.c_int32), ("reserved", C.c_int32), ("t_submit", C.c_double),
                ("t_admit", C.c_double), ("t_complete", C.c_double), ("histories", C.c_uint64),
                ("scatter_counts", C.c_void_p), ("scatter_weights", C.c_void_p)]


class KernelTiming(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("dropped", C.c_uint64), ("transport_ms", C.c_double),
                ("coincidence_ms", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [(k, C.c_uint64) for k in ("submitted", "completed", "cancelled", "ticks", "histories",
                                          "max_active_seen", "bytes_allocated", "budget_bytes", "failed")]


REQ_DONE, REQ_CANCELLED, REQ_FAILED = 0, 1, 2

# every entry point of include/sse.h: name -> (argtypes, restype)
_P = C.c_void_p
SIGNATURES = {
    "sse_abi_version": ([], C.c_int),
    "sse_last_error": ([], C.c_char_p),
    "sse_create": ([C.POINTER(C.c_void_p), C.c_int, _P, _P, _P], C.c_int),
    "sse_destroy": ([_P], C.c_int),
    "sse_load_phantom": ([_P, _P, _P, _P, C.c_int, _P, C.POINTER(C.c_uint32)], C.c_int),
    "sse_update_activity": ([_P, C.c_uint32, _P, C.c_int, _P], C.c_int),
    "sse_unload_phantom": ([_P, C.c_uint32], C.c_int),
    "sse_load_lut": ([_P, _P, _P, C.c_int, C.c_int, _P], C.c_int),
    "sse_load_sensitivity": ([_P, _P, C.c_int, C.c_int, _P], C.c_int),
    "sse_set_gaps": ([_P, _P, _P, _P, C.c_int, _P], C.c_int),
    "sse_set_pair_pruning": ([_P, C.c_int], C.c_int),
    "sse_set_pair_buffer": ([_P, C.c_uint64], C.c_int),
    "sse_build_edge_lut": ([_P, _P], C.c_int),
    "sse_check_division": ([_P, C.c_uint64, C.c_uint32, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64)], C.c_int),
    "sse_simulate": ([_P, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint64, _P, _P], C.c_int),
    "sse_simulate_noalloc": ([_P, C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint64, _P, _P], C.c_int),
    "sse_set_kernel_timing": ([_P, C.c_int, C.c_uint32], C.c_int),
    "sse_read_kernel_timing": ([_P, _P], C.c_int),
    "sse_emission_scale": ([_P, C.c_uint32, C.c_uint64, C.c_double, C.c_double, C.POINTER(C.c_double)], C.c_int),
    "sse_apply_sensitivity": ([_P, _P, C.c_double, _P, _P], C.c_int),
    "sse_total_scatter": ([_P, _P, C.c_double, _P, _P], C.c_int),
    "sse_gaussian_smooth": ([_P, _P, _P, _P, C.c_float, _P], C.c_int),
    "sse_finalize": ([_P, _P, C.c_double, _P, C.c_float, _P, _P], C.c_int),
    "sse_smoothing_normalisation": ([_P, _P, C.c_double, _P, C.c_float, _P, _P], C.c_int),
    "sse_finalize_normalised": ([_P, _P, C.c_double, _P, _P, C.c_float, _P, _P], C.c_int),
    "sse_project": ([_P, C.c_uint32, _P, _P, C.c_int, C.c_int, C.c_int, _P], C.c_int),
    "sse_backproject": ([_P, C.c_uint32, _P, _P, C.c_int, C.c_int, C.c_int, _P], C.c_int),
    "sse_osem": ([_P, C.c_uint32, _P, _P, _P, _P, _P, C.c_int, C.c_int, _P], C.c_int),
    "sse_osem_sensitivity": ([_P, C.c_uint32, _P, C.c_int, _P, _P], C.c_int),
    "sse_image_to_activity": ([_P, C.c_uint32, _P, _P], C.c_int),
    "sse_attenuation_factors": ([_P, C.c_uint32, _P, _P], C.c_int),
    "sse_build_alias_table": ([_P, C.c_uint64, _P, _P], C.c_int),
    "sse_server_start": ([_P, _P, C.POINTER(C.c_void_p)], C.c_int),
    "sse_server_submit": ([_P, _P, C.POINTER(C.c_uint64)], C.c_int),
    "sse_server_poll": ([_P, _P, C.c_int32, C.POINTER(C.c_int32), C.c_int32], C.c_int),
    "sse_server_cancel": ([_P, C.c_uint64], C.c_int),
    "sse_server_release": ([_P, C.c_uint64], C.c_int),
    "sse_server_stats_get": ([_P, _P], C.c_int),
    "sse_server_stop": ([_P], C.c_int),
}

_lib = None


def lib():
    """Load libsse.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2509_05047_amd/build.py "
                              "(or __graft_entry__.build())")
        handle = C.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.argtypes = args
            fn.restype = res
        _lib = handle
    return _lib


def _check(status):
    if status != OK:
        raise SseError(status, lib().sse_last_error().decode())


def _ptr(t):
    """Device or host address of a torch tensor / numpy array (None -> NULL)."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if isinstance(t, np.ndarray):
        return t.ctypes.data
    return t.data_ptr()


def _stream_ptr(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def scanner_desc(s) -> ScannerDesc:
    return ScannerDesc(s.n_crystals, s.n_rings, s.radius_mm, s.length_mm, s.crystals_per_module,
                       s.rings_per_block, s.max_ring_diff)


def sino_desc(s) -> SinoDesc:
    return SinoDesc(s.n_rad, s.n_view, s.n_plane, s.n_tof, s.tof_bin_mm, s.tof_sigma_mm)


def physics_desc(p: dict) -> PhysicsDesc:
    return PhysicsDesc(p["e_lo_kev"], p["e_hi_kev"], p["e_kill_kev"], p["e_fwhm_frac"], p["f_compton"],
                       p["f_rayleigh"], p["f_photo"], p["rayleigh_beta"], p["mu_majorant"], p["max_interactions"])


def build_alias_table(activity: np.ndarray):
    """The library's host alias table for an activity array."""
    a = np.ascontiguousarray(activity, np.float32).ravel()
    th = np.zeros(a.size, np.uint32)
    al = np.zeros(a.size, np.uint32)
    _check(lib().sse_build_alias_table(a.ctypes.data, a.size, th.ctypes.data, al.ctypes.data))
    return th, al


def build_edge_lut(geom) -> np.ndarray:
    """The library's edge-crystal LUT ([angle][position] float32) for a
    mapping with gap_mm, depth_mm, doi_mm, mu_per_mm, n_angle, n_pos."""
    g = EdgeGeom(geom["gap_mm"], geom["depth_mm"], geom["doi_mm"], geom["mu_per_mm"], int(geom["n_angle"]),
                 int(geom["n_pos"]))
    out = np.zeros(max(g.n_angle, 0) * max(g.n_pos, 0), np.float32)
    _check(lib().sse_build_edge_lut(C.byref(g), out.ctypes.data))
    return out.reshape(g.n_angle, g.n_pos)


class Context:
    """A scatter-estimation context on one GPU (see sse_create)."""

    def __init__(self, scanner, sino, physics: dict, device: int = 0):
        self._sc, self._sn, self._ph = scanner_desc(scanner), sino_desc(sino), physics_desc(physics)
        self.sino = sino
        self.scanner = scanner
        self.device = device
        self._grids = {}
        h = C.c_void_p()
        _check(lib().sse_create(C.byref(h), device, C.byref(self._sc), C.byref(self._sn), C.byref(self._ph)))
        self._h = h

    @property
    def n_bins(self) -> int:
        return self.sino.n_rad * self.sino.n_view * self.sino.n_plane * self.sino.n_tof

    def close(self):
        if getattr(self, "_h", None):
            _check(lib().sse_destroy(self._h))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- resources ---------------------------------------------------------
    def load_phantom(self, desc, mu, activity, stream=None) -> int:
        d = PhantomDesc(desc.nx, desc.ny, desc.nz, (C.c_float * 3)(*desc.voxel_mm), (C.c_float * 3)(*desc.lo_mm))
        mem, mu_, act_ = self._as_input(mu, activity)
        pid = C.c_uint32()
        _check(lib().sse_load_phantom(self._h, C.byref(d), _ptr(mu_), _ptr(act_), mem,
                                      _stream_ptr(stream) if mem == MEM_DEVICE else None, C.byref(pid)))
        self._grids[pid.value] = (desc.ny, desc.nx)
        return pid.value

    def phantom_grid(self, pid: int):
        """(ny, nx) of a loaded phantom: the image grid of the reconstruction calls."""
        return self._grids[pid]

    def update_activity(self, pid: int, activity, stream=None):
        mem, act_ = self._as_input(activity)
        _check(lib().sse_update_activity(self._h, pid, _ptr(act_), mem,
                                         _stream_ptr(stream) if mem == MEM_DEVICE else None))

    def unload_phantom(self, pid: int):
        _check(lib().sse_unload_phantom(self._h, pid))

    def load_lut(self, desc, values, dtype: int = F32, stream=None):
        d = LutDesc((C.c_int32 * 5)(*desc.dims), desc.e_min_kev, desc.e_max_kev)
        if isinstance(values, np.ndarray):
            v = np.ascontiguousarray(values)
            want = np.float32 if dtype == F32 else np.uint16
            if v.dtype != want:
                raise TypeError(f"LUT values must be {np.dtype(want)} for dtype {dtype}")
            _check(lib().sse_load_lut(self._h, C.byref(d), v.ctypes.data, dtype, MEM_HOST, None))
        else:
            _check(lib().sse_load_lut(self._h, C.byref(d), _ptr(values.contiguous()), dtype, MEM_DEVICE,
                                      _stream_ptr(stream)))

    def set_gaps(self, gaps=None, edge_t=None, edge_a=None):
        """Gap model on (a mapping with transaxial_gap_rad, axial_gap_mm,
        policy as name or number, edge_n_angle / edge_n_pos for the edge-LUT
        policy; edge LUTs as float32 numpy arrays) or off (gaps=None)."""
        if gaps is None:
            _check(lib().sse_set_gaps(self._h, None, None, None, MEM_HOST, None))
            return
        pol = gaps["policy"]
        pol = GAP_POLICIES[pol] if isinstance(pol, str) else int(pol)
        d = GapDesc(gaps["transaxial_gap_rad"], gaps["axial_gap_mm"], pol, int(gaps.get("edge_n_angle", 0)),
                    int(gaps.get("edge_n_pos", 0)), 0)
        et = None if edge_t is None else np.ascontiguousarray(edge_t, np.float32)
        ea = None if edge_a is None else np.ascontiguousarray(edge_a, np.float32)
        _check(lib().sse_set_gaps(self._h, C.byref(d), _ptr(et), _ptr(ea), MEM_HOST, None))

    def set_pair_buffer(self, max_records: int):
        """Most records of the pair buffer (see sse_set_pair_buffer)."""
        _check(lib().sse_set_pair_buffer(self._h, int(max_records)))

    def set_pair_pruning(self, enable: bool):
        """Do not track photon B when photon A ended outside the energy
        window (sinograms unchanged; see sse_set_pair_pruning)."""
        _check(lib().sse_set_pair_pruning(self._h, 1 if enable else 0))

    def check_division(self, n_random: int = 1 << 30, seed: int = 1):
        """(reciprocal mismatches, quotient mismatches) of the device division
        against the IEEE operator (see sse_check_division); both 0 expected."""
        r, q = C.c_uint64(), C.c_uint64()
        _check(lib().sse_check_division(self._h, n_random, seed, C.byref(r), C.byref(q)))
        return r.value, q.value

    def load_sensitivity(self, sens, has_tof_axis: bool = True, stream=None):
        mem, s_ = self._as_input(sens)
        _check(lib().sse_load_sensitivity(self._h, _ptr(s_), int(has_tof_axis), mem,
                                          _stream_ptr(stream) if mem == MEM_DEVICE else None))

    @staticmethod
    def _as_input(*arrays):
        if all(isinstance(a, np.ndarray) for a in arrays):
            return (MEM_HOST,) + tuple(np.ascontiguousarray(a, np.float32) for a in arrays)
        import torch
        out = []
        for a in arrays:
            if not (isinstance(a, torch.Tensor) and a.is_cuda and a.dtype == torch.float32):
                raise TypeError("inputs must all be numpy float32 arrays or all CUDA float32 tensors")
            out.append(a.contiguous())
        return (MEM_DEVICE,) + tuple(out)

    # -- compute -------------------------------------------------------------
    def new_outputs(self, trues: bool = False, stats: bool = False, records: int = 0, record_stride: int = 1):
        """Zeroed device output tensors for simulate().  Statistics counters
        (stats=True) or per-history records make simulate() run the
        instrumented kernel, which is slower; the default asks for neither."""
        import torch
        dev = torch.device("cuda", self.device)
        o = {"scatter_counts": torch.zeros(self.n_bins, dtype=torch.int32, device=dev),
             "scatter_weights": torch.zeros(self.n_bins, dtype=torch.float64, device=dev)}
        if trues:
            o["true_counts"] = torch.zeros(self.n_bins, dtype=torch.int32, device=dev)
            o["true_weights"] = torch.zeros(self.n_bins, dtype=torch.float64, device=dev)
        if stats:
            o["stats"] = torch.zeros(STAT_COUNT, dtype=torch.int64, device=dev)
        if records:
            o["records"] = torch.zeros((records, RECORD_WORDS), dtype=torch.int32, device=dev)
            o["record_stride"] = record_stride
        return o

    def simulate(self, pid: int, n_histories: int, seed: int, outputs: dict, h_offset: int = 0, stream=None):
        """Accumulate histories [h_offset, h_offset + n) into `outputs` (from new_outputs)."""
        o = Outputs(_ptr(outputs["scatter_counts"]), _ptr(outputs["scatter_weights"]),
                    _ptr(outputs.get("true_counts")), _ptr(outputs.get("true_weights")),
                    _ptr(outputs.get("stats")), _ptr(outputs.get("records")),
                    int(outputs.get("record_stride", 1)) if outputs.get("records") is not None else 0)
        _check(lib().sse_simulate(self._h, pid, n_histories, seed, h_offset, C.byref(o), _stream_ptr(stream)))

    def simulate_noalloc(self, pid: int, n_histories: int, seed: int, outputs: dict, h_offset: int = 0,
                         stream=None):
        """simulate() through the allocation-free entry point (scatter and
        trues sinograms only: no statistics, no records)."""
        o = Outputs(_ptr(outputs["scatter_counts"]), _ptr(outputs["scatter_weights"]),
                    _ptr(outputs.get("true_counts")), _ptr(outputs.get("true_weights")),
                    _ptr(outputs.get("stats")), _ptr(outputs.get("records")),
                    int(outputs.get("record_stride", 1)) if outputs.get("records") is not None else 0)
        _check(lib().sse_simulate_noalloc(self._h, pid, n_histories, seed, h_offset, C.byref(o),
                                          _stream_ptr(stream)))

    def set_kernel_timing(self, enable: bool, max_launches: int = 4096):
        _check(lib().sse_set_kernel_timing(self._h, int(bool(enable)), int(max_launches)))

    def read_kernel_timing(self) -> dict:
        """{launches, dropped, transport_ms, coincidence_ms} since the last read."""
        t = KernelTiming()
        _check(lib().sse_read_kernel_timing(self._h, C.byref(t)))
        return {f[0]: getattr(t, f[0]) for f in KernelTiming._fields_}

    def emission_scale(self, pid: int, n_histories: int, acq_seconds: float = 1.0, factor: float = 1.0) -> float:
        v = C.c_double()
        _check(lib().sse_emission_scale(self._h, pid, n_histories, acq_seconds, factor, C.byref(v)))
        return v.value

    def apply_sensitivity(self, weights, scale: float, out, stream=None):
        _check(lib().sse_apply_sensitivity(self._h, _ptr(weights), scale, _ptr(out), _stream_ptr(stream)))

    # reconstruction (joint estimation loop): images are [n_plane][ny][nx]
    # float32 device tensors on the grid of phantom `grid`
    def project(self, grid: int, image, sino, tof: bool = True, subset: int = 0, n_subsets: int = 1, stream=None):
        _check(lib().sse_project(self._h, grid, _ptr(image), _ptr(sino), int(bool(tof)), subset, n_subsets,
                                 _stream_ptr(stream)))

    def backproject(self, grid: int, sino, image, tof: bool = True, subset: int = 0, n_subsets: int = 1,
                    stream=None):
        _check(lib().sse_backproject(self._h, grid, _ptr(sino), _ptr(image), int(bool(tof)), subset, n_subsets,
                                     _stream_ptr(stream)))

    def osem(self, grid: int, prompts, mult, additive, image, n_iter: int = 1, n_subsets: int = 1, sens=None,
             stream=None):
        """sens: the subset sensitivity images of osem_sensitivity (or None)."""
        _check(lib().sse_osem(self._h, grid, _ptr(prompts), _ptr(mult), _ptr(additive), _ptr(sens), _ptr(image),
                              n_iter, n_subsets, _stream_ptr(stream)))

    def osem_sensitivity(self, grid: int, mult, n_subsets: int, stream=None):
        """The n_subsets subset sensitivity images, a new device tensor."""
        import torch
        ny, nx = self.phantom_grid(grid)
        sens = torch.empty((n_subsets, self.sino.n_plane, ny, nx), dtype=torch.float32,
                           device=torch.device("cuda", self.device))
        _check(lib().sse_osem_sensitivity(self._h, grid, _ptr(mult), n_subsets, _ptr(sens), _stream_ptr(stream)))
        return sens

    def attenuation_factors(self, pid: int, out, stream=None):
        """exp(-line integral of the phantom's attenuation) per LOR, [plane][view][rad]."""
        _check(lib().sse_attenuation_factors(self._h, pid, _ptr(out), _stream_ptr(stream)))

    def image_to_activity(self, pid: int, image, stream=None):
        _check(lib().sse_image_to_activity(self._h, pid, _ptr(image), _stream_ptr(stream)))

    def total_scatter(self, weights, scale: float, stream=None):
        """Binary64 total of scale * W * sens, reduced on the device; returns
        a one-element float64 device tensor."""
        import torch
        t = torch.empty(1, dtype=torch.float64, device=torch.device("cuda", self.device))
        _check(lib().sse_total_scatter(self._h, _ptr(weights), scale, _ptr(t), _stream_ptr(stream)))
        return t

    def gaussian_smooth(self, x, out, sigma_bins, truncate: float = 4.0, stream=None):
        s = (C.c_float * 3)(*sigma_bins)
        _check(lib().sse_gaussian_smooth(self._h, _ptr(x), _ptr(out), s, truncate, _stream_ptr(stream)))

    def finalize(self, weights, scale: float, out, sigma_bins=None, truncate: float = 4.0, stream=None):
        s = None if sigma_bins is None else (C.c_float * 3)(*sigma_bins)
        _check(lib().sse_finalize(self._h, _ptr(weights), scale, s, truncate, _ptr(out), _stream_ptr(stream)))

    def smoothing_normalisation(self, weights, scale: float, out, sigma_bins, truncate: float = 4.0, stream=None):
        """out = G_heavy(S) / S (1 where undefined), S = float(scale * weights)."""
        s = (C.c_float * 3)(*sigma_bins)
        _check(lib().sse_smoothing_normalisation(self._h, _ptr(weights), scale, s, truncate, _ptr(out),
                                                 _stream_ptr(stream)))

    def finalize_normalised(self, weights, scale: float, norm, out, sigma_bins, truncate: float = 4.0,
                            stream=None):
        """out = sens * G(S * norm) / norm, S = float(scale * weights)."""
        s = (C.c_float * 3)(*sigma_bins)
        _check(lib().sse_finalize_normalised(self._h, _ptr(weights), scale, _ptr(norm), s, truncate, _ptr(out),
                                             _stream_ptr(stream)))


def stats_dict(t) -> dict:
    """Statistics tensor -> {name: int}."""
    v = t.cpu().numpy().astype(np.uint64)
    return {k: int(x) for k, x in zip(STAT_NAMES, v)}


class Server:
    """Request server on a context (see sse_server_start): continuous
    batching of scatter-estimate requests with HBM-footprint admission."""

    def __init__(self, ctx: Context, max_active: int = 16, hbm_budget_bytes: int = 0, tick_histories: int = 0,
                 chunk_histories: int = 0):
        self.ctx = ctx
        cfg = ServerCfg(max_active, 0, int(hbm_budget_bytes), int(tick_histories), int(chunk_histories))
        h = C.c_void_p()
        _check(lib().sse_server_start(ctx._h, C.byref(cfg), C.byref(h)))
        self._h = h

    def submit(self, pid: int, n_histories: int, seed: int, h_offset: int = 0, counts=None, weights=None) -> int:
        r = Request(pid, 0, int(n_histories), int(seed), int(h_offset), _ptr(counts), _ptr(weights))
        rid = C.c_uint64()
        _check(lib().sse_server_submit(self._h, C.byref(r), C.byref(rid)))
        return rid.value

    def poll(self, max_n: int = 64, wait_ms: int = 0) -> list:
        buf = (Completion * max_n)()
        n = C.c_int32()
        _check(lib().sse_server_poll(self._h, buf, max_n, C.byref(n), int(wait_ms)))
        return [{f[0]: getattr(buf[i], f[0]) for f in Completion._fields_} for i in range(n.value)]

    def cancel(self, rid: int):
        _check(lib().sse_server_cancel(self._h, rid))

    def release(self, rid: int):
        _check(lib().sse_server_release(self._h, rid))

    def stats(self) -> dict:
        st = ServerStats()
        _check(lib().sse_server_stats_get(self._h, C.byref(st)))
        return {f[0]: getattr(st, f[0]) for f in ServerStats._fields_}

    def stop(self):
        if getattr(self, "_h", None):
            h, self._h = self._h, None
            _check(lib().sse_server_stop(h))

    def __del__(self):
        try:
            self.stop()
        except Exception:
            pass


def copy_device_to_tensor(ptr: int, n: int, dtype):
    """Copy n elements at a device address into a new torch tensor (used for
    server-allocated results)."""
    import torch
    out = torch.empty(n, dtype=dtype, device="cuda")
    hip = C.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
    hip.hipMemcpy.restype = C.c_int
    err = hip.hipMemcpy(out.data_ptr(), ptr, n * out.element_size(), 3)  # device to device
    if err != 0:
        raise SseError(EDEVICE, f"hipMemcpy failed ({err})")
    return out
