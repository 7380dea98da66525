"""Python binding of the C ABI in include/omc.h (argument marshalling only).

Every step of the transport runs in the HIP library ``_lib/libomc.so``; this
module only converts numpy arrays, dictionaries and torch device buffers into
the plain pointers and structs the C functions take. If the library is not
built, loading fails with an error: there is no fallback path.
"""
import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libomc.so")

OMC_OK, OMC_EINVAL, OMC_ENOMEM, OMC_EDEVICE, OMC_ESTATE, OMC_EQUEUE, OMC_ENUMERIC, OMC_EUNSUP = (
    0, -1, -2, -3, -4, -5, -6, -7)
NE = 512
NA = 512
TABLE_ROWS = ["muC", "muPE", "muPair", "muTot", "Scol", "Srad", "R", "sigM", "sigB", "sigHat",
              "K1"]
EXPORTS = ["omc_default_params", "omc_create", "omc_set_phantom", "omc_set_phantom_ct",
           "omc_get_phantom",
           "omc_set_source",
           "omc_set_params",
           "omc_get_params", "omc_get_geometry", "omc_run", "omc_run_device",
           "omc_run_device_static", "omc_run_beamlets", "omc_free_sparse",
           "omc_autotune", "omc_get_counters", "omc_get_timing", "omc_debug_philox",
           "omc_debug_trace", "omc_debug_sample", "omc_host_tables", "omc_host_ms_table", "omc_last_error",
           "omc_destroy",
           # include/omc_dn.h
           "omc_dn_create", "omc_dn_num_params", "omc_dn_get_params", "omc_dn_set_params",
           "omc_dn_forward", "omc_dn_train_step", "omc_dn_gradient", "omc_dn_denoise",
           "omc_dn_debug_layer", "omc_dn_last_error", "omc_dn_destroy"]
VOID_FNS = ("omc_default_params", "omc_last_error", "omc_destroy", "omc_free_sparse",
            "omc_dn_last_error", "omc_dn_destroy")


class OmcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"omc error {code}: {msg}")
        self.code = code


class Material(C.Structure):
    _fields_ = [("n_elem", C.c_int), ("Z", C.POINTER(C.c_int)), ("A", C.POINTER(C.c_double)),
                ("w_mass", C.POINTER(C.c_double)), ("I_eV", C.c_double),
                ("rho_nominal", C.c_double)]


class Source(C.Structure):
    _fields_ = [("particle", C.c_int), ("n_bins", C.c_int), ("edges", C.POINTER(C.c_double)),
                ("weights", C.POINTER(C.c_double)), ("mono_E", C.c_double),
                ("geometry", C.c_int), ("ssd", C.c_double), ("z_field", C.c_double),
                ("fx", C.c_double), ("fy", C.c_double), ("cx", C.c_double), ("cy", C.c_double),
                ("sx", C.c_double), ("sy", C.c_double), ("gantry_deg", C.c_double),
                ("iso_x", C.c_double), ("iso_z", C.c_double),
                ("n_psf", C.c_int), ("psf", C.POINTER(C.c_float)), ("psf_on_device", C.c_int)]


class CtMap(C.Structure):
    _fields_ = [("n_nodes", C.c_int), ("hu", C.POINTER(C.c_double)), ("rho", C.POINTER(C.c_double)),
                ("n_bins", C.c_int), ("hu_upper", C.POINTER(C.c_double)),
                ("material", C.POINTER(C.c_int))]


class Params(C.Structure):
    _fields_ = [("Eabs_e", C.c_double), ("Eabs_g", C.c_double), ("Wcc", C.c_double),
                ("kc", C.c_double), ("dmax_s", C.c_double), ("f_E", C.c_double),
                ("n_batches", C.c_int), ("parity_fp64", C.c_int), ("kerma_mode", C.c_int),
                ("csda_mode", C.c_int), ("block_size", C.c_int), ("blocks_per_cu", C.c_int),
                ("chunk_histories", C.c_int), ("queue_factor", C.c_int), ("timing", C.c_int),
                ("graph_depth", C.c_int), ("beamlet_group", C.c_int),
                ("sparse_threshold", C.c_double), ("straggler_lanes", C.c_int),
                ("electron_mode", C.c_int), ("table_mode", C.c_int), ("photon_mode", C.c_int),
                ("tally_copies", C.c_int), ("source_order", C.c_int),
                ("event_lanes", C.c_int)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Beamlet(C.Structure):
    _fields_ = [("src", Source), ("n_histories", C.c_uint64), ("h0", C.c_uint32)]


class SparseOut(C.Structure):
    _fields_ = [("n_beamlets", C.c_int), ("on_device", C.c_int), ("nnz", C.c_uint64),
                ("row_ptr", C.POINTER(C.c_uint64)), ("voxel", C.POINTER(C.c_uint32)),
                ("dose", C.POINTER(C.c_float))]


COUNTER_INT = ["ph_flights", "ph_fictitious", "ph_compton", "ph_photo", "ph_pair", "ph_cutoff",
               "ph_escaped", "el_steps", "el_hard_cand", "el_hard_fict", "el_moller", "el_brems",
               "el_absorbed", "el_escaped", "el_boundary", "el_hinge_trunc", "pos_annihil",
               "push_ph", "push_el", "src_miss"]
COUNTER_EXTRA = ["watchdog"]
COUNTER_FP = ["E_incident", "E_deposited", "E_escaped", "E_pair_rest", "E_annih_rest"]


class Counters(C.Structure):
    _fields_ = ([(n, C.c_uint64) for n in COUNTER_INT + COUNTER_EXTRA]
                + [(n, C.c_double) for n in COUNTER_FP]
                + [("queue_hwm_ph", C.c_uint64), ("queue_hwm_el", C.c_uint64),
                   ("iterations", C.c_uint32), ("max_steps", C.c_uint32),
                   ("set_aside", C.c_uint64)])

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class Timing(C.Structure):
    _fields_ = [("launches", C.c_uint32 * 4), ("total_ms", C.c_double * 4), ("run_ms", C.c_double),
                ("tables_global", C.c_int)]

    def as_dict(self):
        names = ["source", "photon", "electron", "fold"]
        return {"launches": dict(zip(names, list(self.launches))),
                "total_ms": dict(zip(names, list(self.total_ms))), "run_ms": self.run_ms,
                "tables_global": self.tables_global}


_lib = None


def lib():
    """Load the HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library {LIB_PATH} is not built; run "
                               "`python -c 'import __graft_entry__ as g; g.build()'`")
        # torch ships its own HIP runtime with the same soname; loading torch
        # first makes this library bind to it, so that device pointers and
        # streams from torch are valid here (one runtime per process)
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        dp = C.POINTER(C.c_double)
        L.omc_default_params.argtypes = [C.POINTER(Params)]
        L.omc_default_params.restype = None
        L.omc_create.argtypes = [C.POINTER(vp), C.c_int, C.c_int, C.c_int, C.c_double, C.c_double,
                                 C.c_double, C.POINTER(C.c_float), C.POINTER(C.c_uint8),
                                 C.POINTER(Material), C.c_int]
        L.omc_set_phantom.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_uint8)]
        L.omc_set_phantom_ct.argtypes = [vp, vp, C.c_int, C.POINTER(CtMap)]
        L.omc_get_phantom.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_uint8)]
        L.omc_set_source.argtypes = [vp, C.POINTER(Source)]
        L.omc_set_params.argtypes = [vp, C.POINTER(Params)]
        L.omc_get_params.argtypes = [vp, C.POINTER(Params)]
        L.omc_debug_sample.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.c_uint32,
                                       C.c_uint32, C.POINTER(C.c_double),
                                       C.POINTER(C.c_uint32)]
        ip = C.POINTER(C.c_int)
        dp_ = C.POINTER(C.c_double)
        L.omc_get_geometry.argtypes = [vp, ip, ip, ip, dp_, dp_, dp_]
        L.omc_run.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, dp, dp]
        L.omc_run_device.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, vp, vp, vp]
        L.omc_run_device_static.argtypes = [vp, C.c_uint64, C.c_uint32, C.c_uint32, vp, vp, vp]
        L.omc_run_beamlets.argtypes = [vp, C.POINTER(Beamlet), C.c_int, C.c_uint32, C.c_int, vp,
                                       C.POINTER(SparseOut)]
        L.omc_free_sparse.argtypes = [C.POINTER(SparseOut)]
        L.omc_free_sparse.restype = None
        L.omc_autotune.argtypes = [vp, C.c_uint64, C.c_uint32, C.POINTER(Params)]
        L.omc_get_counters.argtypes = [vp, C.POINTER(Counters)]
        L.omc_get_timing.argtypes = [vp, C.POINTER(Timing)]
        L.omc_debug_philox.argtypes = [C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint32,
                                       C.POINTER(C.c_uint32)]
        L.omc_debug_trace.argtypes = [vp, C.c_uint32, C.c_uint32, dp, C.c_uint32,
                                      C.POINTER(C.c_uint32)]
        L.omc_host_tables.argtypes = [C.POINTER(Material), C.c_double, C.c_double, dp]
        L.omc_host_ms_table.argtypes = [dp]
        L.omc_last_error.argtypes = [vp]
        L.omc_last_error.restype = C.c_char_p
        L.omc_destroy.argtypes = [vp]
        L.omc_destroy.restype = None
        fp = C.POINTER(C.c_float)
        L.omc_dn_create.argtypes = [C.POINTER(vp), C.c_int, C.c_int, C.c_int, C.c_uint32]
        L.omc_dn_num_params.argtypes = [vp, C.POINTER(C.c_uint64)]
        L.omc_dn_get_params.argtypes = [vp, fp, C.c_uint64]
        L.omc_dn_set_params.argtypes = [vp, fp, C.c_uint64]
        L.omc_dn_forward.argtypes = [vp, vp, vp, vp, C.c_double, vp, vp]
        L.omc_dn_train_step.argtypes = [vp, vp, vp, vp, C.c_double, vp, C.c_double, fp, vp]
        L.omc_dn_gradient.argtypes = [vp, vp, vp, vp, C.c_double, vp, fp, C.c_uint64, fp, vp]
        L.omc_dn_denoise.argtypes = [vp, vp, C.c_uint64, C.c_uint32, C.c_uint32, vp, C.c_double,
                                     C.c_uint64, vp, dp, C.POINTER(C.c_int), vp]
        L.omc_dn_debug_layer.argtypes = [C.c_int] * 7 + [fp] * 8
        L.omc_dn_last_error.argtypes = [vp]
        L.omc_dn_last_error.restype = C.c_char_p
        L.omc_dn_destroy.argtypes = [vp]
        L.omc_dn_destroy.restype = None
        for name in EXPORTS:
            if name not in VOID_FNS:
                getattr(L, name).restype = C.c_int
        _lib = L
    return _lib


def _check(rc, ctx=None):
    if rc != OMC_OK:
        msg = lib().omc_last_error(ctx)
        raise OmcError(rc, msg.decode() if msg else "")


def _dptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class _MaterialHolder:
    def __init__(self, spec):
        self.Z = np.ascontiguousarray(spec["Z"], dtype=np.int32)
        self.A = np.ascontiguousarray(spec["A"], dtype=np.float64)
        self.w = np.ascontiguousarray(spec["w"], dtype=np.float64)
        self.struct = Material(len(self.Z), self.Z.ctypes.data_as(C.POINTER(C.c_int)),
                               _dptr(self.A), _dptr(self.w), float(spec["I_eV"]),
                               float(spec["rho_nom"]))


def default_params():
    p = Params()
    lib().omc_default_params(C.byref(p))
    return p


class Engine:
    """One phantom on the current HIP device (see omc_create)."""

    def __init__(self, phantom):
        """phantom: {"shape" (z, y, x), "voxel", "materials", and either "density"
        and "material" arrays or a CT volume "hu" with its "ct_map" (mapped on
        the device by omc_set_phantom_ct)."""
        self.shape = tuple(phantom["shape"])
        nz, ny, nx = self.shape
        dz, dy, dx = phantom["voxel"]
        ct = "density" not in phantom and "hu" in phantom
        if ct:
            dens = np.ones(nz * ny * nx, np.float32)
            mat = np.zeros(nz * ny * nx, np.uint8)
        else:
            dens = np.ascontiguousarray(phantom["density"], dtype=np.float32).ravel()
            mat = np.ascontiguousarray(phantom["material"], dtype=np.uint8).ravel()
        # materials None: the library's built-in water, lung and bone
        mats = phantom.get("materials")
        holders = [_MaterialHolder(m) for m in mats] if mats is not None else []
        arr = (Material * len(holders))(*[h.struct for h in holders]) if holders else None
        h = C.c_void_p()
        rc = lib().omc_create(C.byref(h), nx, ny, nz, dx, dy, dz,
                              dens.ctypes.data_as(C.POINTER(C.c_float)),
                              mat.ctypes.data_as(C.POINTER(C.c_uint8)), arr, len(holders))
        _check(rc, None)
        self._h = h
        self.params = default_params()
        if ct:
            self.set_phantom_ct(phantom["hu"], phantom["ct_map"])

    def close(self):
        if getattr(self, "_h", None):
            lib().omc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_phantom(self, phantom):
        """New densities and materials for the same dimensions (omc_set_phantom)."""
        assert tuple(phantom["shape"]) == self.shape
        dens = np.ascontiguousarray(phantom["density"], dtype=np.float32).ravel()
        mat = np.ascontiguousarray(phantom["material"], dtype=np.uint8).ravel()
        _check(lib().omc_set_phantom(self._h, dens.ctypes.data_as(C.POINTER(C.c_float)),
                                     mat.ctypes.data_as(C.POINTER(C.c_uint8))), self._h)

    def set_phantom_ct(self, hu, ct_map):
        """Densities and materials from a CT volume (omc_set_phantom_ct): hu is an
        int16 array of the phantom's shape (z, y, x), on the host or a device
        tensor; ct_map a dict with "hu", "rho" (calibration nodes), "upper" (bin
        upper bounds) and "material" (library id per bin)."""
        nodes = np.ascontiguousarray(ct_map["hu"], dtype=np.float64)
        rho = np.ascontiguousarray(ct_map["rho"], dtype=np.float64)
        upper = np.ascontiguousarray(ct_map["upper"], dtype=np.float64)
        mats = np.ascontiguousarray(ct_map["material"], dtype=np.int32)
        if len(nodes) != len(rho) or len(upper) != len(mats):
            raise ValueError("ct_map: hu/rho and upper/material must pair up")
        m = CtMap(len(nodes), _dptr(nodes), _dptr(rho), len(mats), _dptr(upper),
                  mats.ctypes.data_as(C.POINTER(C.c_int)))
        if getattr(hu, "is_cuda", False):
            import torch
            if hu.dtype != torch.int16 or not hu.is_contiguous() or \
                    tuple(hu.shape) != self.shape:
                raise ValueError("device HU must be a contiguous int16 tensor of the phantom's "
                                 "shape")
            ptr, on_dev = C.c_void_p(hu.data_ptr()), 1
        else:
            hu = np.ascontiguousarray(hu, dtype=np.int16)
            if hu.shape != self.shape:
                raise ValueError("HU volume must have the phantom's shape")
            ptr, on_dev = hu.ctypes.data_as(C.c_void_p), 0
        _check(lib().omc_set_phantom_ct(self._h, ptr, on_dev, C.byref(m)), self._h)

    def get_phantom(self):
        """The phantom's densities and material ids as the device holds them
        (omc_get_phantom), shaped (z, y, x)."""
        n = int(np.prod(self.shape))
        dens = np.zeros(n, np.float32)
        mat = np.zeros(n, np.uint8)
        _check(lib().omc_get_phantom(self._h, dens.ctypes.data_as(C.POINTER(C.c_float)),
                                     mat.ctypes.data_as(C.POINTER(C.c_uint8))), self._h)
        return dens.reshape(self.shape), mat.reshape(self.shape)

    def set_source(self, src):
        s, keep = _source_struct(src)
        _check(lib().omc_set_source(self._h, C.byref(s)), self._h)
        # device records are read in place by every run: hold them until the
        # next source replaces them
        self._device_records = keep[2] if s.psf_on_device else None

    def set_params(self, **kw):
        p = Params.from_buffer_copy(self.params)
        for k, v in kw.items():
            setattr(p, k, v)
        _check(lib().omc_set_params(self._h, C.byref(p)), self._h)
        self.params = p

    def run(self, n, seed=1, h0=0, check=True):
        nvox = int(np.prod(self.shape))
        dose = np.zeros(nvox)
        dose2 = np.zeros(nvox)
        rc = lib().omc_run(self._h, int(n), int(seed), int(h0), _dptr(dose), _dptr(dose2))
        if check:
            _check(rc, self._h)
        return dose.reshape(self.shape), dose2.reshape(self.shape)

    def run_device(self, n, seed, h0, dose, dose2, stream=None):
        """dose, dose2: float64 CUDA tensors with nvox elements; stream: a
        torch.cuda.Stream or None for the current stream."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        assert dose.dtype == torch.float64 and dose.is_cuda and dose.is_contiguous()
        assert dose2.dtype == torch.float64 and dose2.is_cuda and dose2.is_contiguous()
        assert dose.numel() == dose2.numel() == int(np.prod(self.shape))
        rc = lib().omc_run_device(self._h, int(n), int(seed), int(h0), C.c_void_p(dose.data_ptr()),
                                  C.c_void_p(dose2.data_ptr()), C.c_void_p(stream.cuda_stream))
        _check(rc, self._h)

    def run_device_static(self, n, seed, h0, dose, dose2, stream=None):
        """As run_device, through omc_run_device_static: the run allocates no
        device memory (the library's fixed scratch; see include/omc.h)."""
        import torch
        if stream is None:
            stream = torch.cuda.current_stream()
        assert dose.dtype == torch.float64 and dose.is_cuda and dose.is_contiguous()
        assert dose2.dtype == torch.float64 and dose2.is_cuda and dose2.is_contiguous()
        assert dose.numel() == dose2.numel() == int(np.prod(self.shape))
        rc = lib().omc_run_device_static(self._h, int(n), int(seed), int(h0),
                                         C.c_void_p(dose.data_ptr()), C.c_void_p(dose2.data_ptr()),
                                         C.c_void_p(stream.cuda_stream))
        _check(rc, self._h)

    def run_beamlets(self, beamlets, seed=1, on_device=False, stream=None):
        """beamlets: list of (source dict, n_histories, h0). Returns a Sparse
        holding the CSR rows (see omc_run_beamlets); host rows unless on_device."""
        arr = (Beamlet * len(beamlets))()
        keep, cache = [], {}
        for i, (src, n, h0) in enumerate(beamlets):
            s, k = _source_struct(src, cache)
            keep.append(k)
            arr[i] = Beamlet(s, int(n), int(h0))
        out = SparseOut()
        sp = None
        if on_device:
            import torch
            sp = (stream or torch.cuda.current_stream()).cuda_stream
        rc = lib().omc_run_beamlets(self._h, arr, len(beamlets), int(seed), int(bool(on_device)),
                                    C.c_void_p(sp), C.byref(out))
        _check(rc, self._h)
        return Sparse(out)

    def autotune(self, n_probe, seed=1):
        """Pick the launch shape by timing (omc_autotune); returns the chosen
        parameters as a dict and applies them."""
        p = Params()
        _check(lib().omc_autotune(self._h, int(n_probe), int(seed), C.byref(p)), self._h)
        self.params = p
        return p.as_dict()

    def trace(self, h, seed=1, max_records=1 << 16):
        """Step records of history h alone (see omc_debug_trace)."""
        out = np.zeros(max_records * 12)
        n = C.c_uint32(0)
        _check(lib().omc_debug_trace(self._h, int(seed), int(h), _dptr(out), max_records,
                                     C.byref(n)), self._h)
        return out[: n.value * 12].reshape(n.value, 12)

    SAMPLERS = {"compton": 0, "moller": 1, "brems": 2, "ms": 3, "annihilation": 4, "pair": 5,
                "source": 6}

    def debug_sample(self, which, args, n, seed=1):
        """n samples of one interaction on the GPU (omc_debug_sample):
        (records (n, 16), stream words used (n,))."""
        a = np.zeros(8)
        a[: len(args)] = args
        out = np.zeros(16 * n)
        words = np.zeros(n, dtype=np.uint32)
        _check(lib().omc_debug_sample(self._h, self.SAMPLERS[which], _dptr(a), int(seed), int(n),
                                      _dptr(out), words.ctypes.data_as(C.POINTER(C.c_uint32))),
               self._h)
        return out.reshape(n, 16), words

    def geometry(self):
        """(nx, ny, nz) voxels and (dx, dy, dz) cm of the context's phantom."""
        n = [C.c_int(0) for _ in range(3)]
        h = [C.c_double(0) for _ in range(3)]
        _check(lib().omc_get_geometry(self._h, *[C.byref(v) for v in n + h]), self._h)
        return tuple(v.value for v in n), tuple(v.value for v in h)

    def get_params(self):
        p = Params()
        _check(lib().omc_get_params(self._h, C.byref(p)), self._h)
        return p.as_dict()

    def counters(self):
        c = Counters()
        _check(lib().omc_get_counters(self._h, C.byref(c)), self._h)
        return c.as_dict()

    def timing(self):
        t = Timing()
        _check(lib().omc_get_timing(self._h, C.byref(t)), self._h)
        return t.as_dict()


def _source_struct(src, cache=None):
    """omc_source for a source dict, and the arrays it points into (keep them
    alive during the call). Equal spectrum arrays share one buffer, and so do
    equal phase-space record arrays."""
    nb = int(src.get("n_bins", 0) or 0)
    key = (id(src.get("edges")), id(src.get("weights")), nb)
    if cache is not None and key in cache:
        edges, weights = cache[key]
    else:
        edges = np.ascontiguousarray(src.get("edges", np.zeros(1)), dtype=np.float64)
        weights = np.ascontiguousarray(src.get("weights", np.zeros(1)), dtype=np.float64)
        if cache is not None:
            cache[key] = (edges, weights)
    recs = src.get("psf")
    n_psf = 0
    psf = None
    on_device = 0
    if recs is not None and getattr(recs, "is_cuda", False):
        # records a caller's GPU code wrote (a torch tensor): read in place
        import torch
        if recs.dtype != torch.float32 or recs.dim() != 2 or recs.shape[1] != 8 \
                or not recs.is_contiguous():
            raise ValueError("device phase-space records must be a contiguous float32 "
                             "tensor of shape (n, 8)")
        psf, n_psf, on_device = recs, int(recs.shape[0]), 1
    elif recs is not None:
        pkey = ("psf", id(recs))
        if cache is not None and pkey in cache:
            psf = cache[pkey]
        else:
            psf = np.ascontiguousarray(recs, dtype=np.float32).reshape(-1, 8)
            if cache is not None:
                cache[pkey] = psf
        n_psf = int(psf.shape[0])
    s = Source(int(src["particle"]), nb, _dptr(edges), _dptr(weights),
               float(src.get("mono_E", 0.0)), int(src["geometry"]),
               float(src.get("ssd", 100.0)), float(src.get("z_field", 0.0)),
               float(src["fx"]), float(src["fy"]), float(src["cx"]), float(src["cy"]),
               float(src.get("sx", src["cx"])), float(src.get("sy", src["cy"])),
               float(src.get("gantry_deg", 0.0)), float(src.get("iso_x", 0.0)),
               float(src.get("iso_z", 0.0)), n_psf,
               (C.cast(C.c_void_p(psf.data_ptr()), C.POINTER(C.c_float)) if on_device else
                psf.ctypes.data_as(C.POINTER(C.c_float)) if psf is not None else None),
               on_device)
    return s, (edges, weights, psf)


class Sparse:
    """CSR rows of omc_run_beamlets; host rows are copied into numpy arrays."""

    def __init__(self, out):
        self._out = out
        self.n_beamlets = out.n_beamlets
        self.nnz = int(out.nnz)
        self.on_device = bool(out.on_device)
        self.row_ptr = (np.ctypeslib.as_array(out.row_ptr, (self.n_beamlets + 1,)).copy()
                        if out.row_ptr else np.zeros(self.n_beamlets + 1, np.uint64))
        if not self.on_device and self.nnz:
            self.voxel = np.ctypeslib.as_array(out.voxel, (self.nnz,)).copy()
            self.dose = np.ctypeslib.as_array(out.dose, (self.nnz,)).copy()
            self.free()
        elif not self.on_device:
            self.voxel = np.zeros(0, np.uint32)
            self.dose = np.zeros(0, np.float32)
            self.free()

    def row(self, b, nvox):
        """Dense dose of beamlet b (host rows only)."""
        d = np.zeros(nvox, np.float64)
        lo, hi = int(self.row_ptr[b]), int(self.row_ptr[b + 1])
        d[self.voxel[lo:hi]] = self.dose[lo:hi]
        return d

    def free(self):
        if self._out is not None:
            lib().omc_free_sparse(C.byref(self._out))
            self._out = None

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


def debug_philox(seed, h, q, n0, nblocks):
    out = np.zeros(4 * nblocks, dtype=np.uint32)
    _check(lib().omc_debug_philox(seed, h, q, n0, nblocks,
                                  out.ctypes.data_as(C.POINTER(C.c_uint32))))
    return out


def host_tables(spec, Wcc=0.05, kc=0.2):
    m = _MaterialHolder(spec)
    out = np.zeros(len(TABLE_ROWS) * NE)
    _check(lib().omc_host_tables(C.byref(m.struct), Wcc, kc, _dptr(out)))
    out = out.reshape(len(TABLE_ROWS), NE)
    return {n: out[i] for i, n in enumerate(TABLE_ROWS)}


def host_ms_table():
    out = np.zeros(NA)
    _check(lib().omc_host_ms_table(_dptr(out)))
    return out


# ------------------------------------------------------------------ denoiser
def _dn_check(rc, h=None):
    if rc != OMC_OK:
        msg = lib().omc_dn_last_error(h)
        raise OmcError(rc, msg.decode() if msg else "")


def _fptr(a):
    return a.ctypes.data_as(C.POINTER(C.c_float)) if a is not None else None


def _dev(t, n=None):
    """Device pointer of a contiguous float32 CUDA tensor (checked)."""
    import torch
    assert t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()
    if n is not None:
        assert t.numel() == n
    return C.c_void_p(t.data_ptr())


class Denoiser:
    """The learned denoiser of include/omc_dn.h for volumes of `shape` (z, y, x)."""

    def __init__(self, shape, seed=0):
        self.shape = tuple(int(k) for k in shape)
        nz, ny, nx = self.shape
        h = C.c_void_p()
        _dn_check(lib().omc_dn_create(C.byref(h), nx, ny, nz, int(seed)))
        self._h = h
        n = C.c_uint64()
        _dn_check(lib().omc_dn_num_params(self._h, C.byref(n)), self._h)
        self.n_params = n.value
        self.nvox = nz * ny * nx

    def close(self):
        if getattr(self, "_h", None):
            lib().omc_dn_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def get_params(self):
        out = np.zeros(self.n_params, np.float32)
        _dn_check(lib().omc_dn_get_params(self._h, _fptr(out), self.n_params), self._h)
        return out

    def set_params(self, theta):
        t = np.ascontiguousarray(theta, dtype=np.float32)
        _dn_check(lib().omc_dn_set_params(self._h, _fptr(t), t.size), self._h)

    def _stream(self, stream):
        import torch
        return C.c_void_p((stream or torch.cuda.current_stream()).cuda_stream)

    def forward(self, dose, sigma, rho, dmax, out, stream=None):
        _dn_check(lib().omc_dn_forward(self._h, _dev(dose, self.nvox), _dev(sigma, self.nvox),
                                       _dev(rho, self.nvox), float(dmax), _dev(out, self.nvox),
                                       self._stream(stream)), self._h)

    def train_step(self, dose, sigma, rho, dmax, target, lr, stream=None):
        loss = C.c_float()
        _dn_check(lib().omc_dn_train_step(self._h, _dev(dose, self.nvox), _dev(sigma, self.nvox),
                                          _dev(rho, self.nvox), float(dmax),
                                          _dev(target, self.nvox), float(lr), C.byref(loss),
                                          self._stream(stream)), self._h)
        return loss.value

    def gradient(self, dose, sigma, rho, dmax, target, stream=None):
        g = np.zeros(self.n_params, np.float32)
        loss = C.c_float()
        _dn_check(lib().omc_dn_gradient(self._h, _dev(dose, self.nvox), _dev(sigma, self.nvox),
                                        _dev(rho, self.nvox), float(dmax),
                                        _dev(target, self.nvox), _fptr(g), self.n_params,
                                        C.byref(loss), self._stream(stream)), self._h)
        return g, loss.value

    def denoise(self, engine, n_low, seed, h0, rho, max_err, n_fallback, out, stream=None):
        err = C.c_double()
        fb = C.c_int()
        _dn_check(lib().omc_dn_denoise(self._h, engine._h, int(n_low), int(seed), int(h0),
                                       _dev(rho, self.nvox), float(max_err), int(n_fallback),
                                       _dev(out, self.nvox), C.byref(err), C.byref(fb),
                                       self._stream(stream)), self._h)
        return err.value, bool(fb.value)


def dn_debug_layer(geometry, x, w, b, gy, c0, c1, want=("y", "gx", "gw", "gb")):
    """One layer on the GPU (omc_dn_debug_layer). x: [z, y, x, c0 + c1], w:
    [taps, c0 + c1, cout] float32; gy: output gradient [z', y', x', cout]."""
    x = np.ascontiguousarray(x, np.float32)
    w = np.ascontiguousarray(w, np.float32)
    nz, ny, nx, cin = x.shape
    cout = w.shape[-1]
    if geometry == 0:
        oshape = (nz, ny, nx)
    elif geometry == 1:
        oshape = (nz // 2, ny // 2, nx // 2)
    else:
        oshape = (2 * nz, 2 * ny, 2 * nx)
    no = int(np.prod(oshape))
    b = np.ascontiguousarray(b, np.float32)
    gy = np.ascontiguousarray(gy, np.float32) if gy is not None else None
    y = np.zeros(no * cout, np.float32) if "y" in want else None
    gx = np.zeros(x.size, np.float32) if "gx" in want else None
    gw = np.zeros(w.size, np.float32) if "gw" in want else None
    gb = np.zeros(cout, np.float32) if "gb" in want else None
    rc = lib().omc_dn_debug_layer(geometry, nx, ny, nz, c0, c1, cout, _fptr(x), _fptr(w), _fptr(b),
                                  _fptr(gy), _fptr(y), _fptr(gx), _fptr(gw), _fptr(gb))
    _dn_check(rc)
    res = {}
    if y is not None:
        res["y"] = y.reshape(oshape + (cout,))
    if gx is not None:
        res["gx"] = gx.reshape(x.shape)
    if gw is not None:
        res["gw"] = gw.reshape(w.shape)
    if gb is not None:
        res["gb"] = gb
    return res
