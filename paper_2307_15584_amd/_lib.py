"""ctypes loader for libqmc.so (the in-tree HIP library).  Fails loudly if it is missing."""

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqmc.so")

QMC_OK = 0
STATUS_NAMES = {
    0: "QMC_OK",
    1: "QMC_ERR_INVALID_ARGUMENT",
    2: "QMC_ERR_OUT_OF_RANGE",
    3: "QMC_ERR_UNSUPPORTED",
    4: "QMC_ERR_DEVICE",
    5: "QMC_ERR_WORKSPACE",
}

QMC_MAX_DIMS = 64
QMC_MAX_DEGREE = 16
QMC_SHIFT_XOR = 1
QMC_LATTICE_BACKWARD = 2
QMC_POINT_MAJOR = 128
QMC_PIXEL_NUS = 4
QMC_PIXEL_SHIFT = 8
QMC_PIXEL_RANDOM_GENERATOR = 16
QMC_PIXEL_HILBERT_SHIFT = 32
QMC_LATTICE_INSTANCES4 = 64
QMC_HALTON_IDENTITY = 0
QMC_HALTON_FAURE = 1
QMC_HALTON_LINEAR = 2
QMC_SAMPLER_SOBOL = 1
QMC_SAMPLER_LATTICE = 2
QMC_SAMPLER_POINTS = 3
QMC_SAMPLER_XOR_TABLE = 4
QMC_PIXEL_TABLE_SHIFT = 256
QMC_XOR_TABLE_CELLS = 16384
QMC_F_GENZ = 1
QMC_F_LOBES = 2
QMC_STATIC_SCRATCH_BYTES = 4 << 20


class Sampler(ctypes.Structure):
    """Mirror of qmc_sampler."""
    _fields_ = [("kind", ctypes.c_uint32), ("s", ctypes.c_uint32), ("table", ctypes.c_void_p),
                ("points_ld", ctypes.c_uint64), ("offsets", ctypes.c_void_p), ("seed", ctypes.c_uint32),
                ("flags", ctypes.c_uint32), ("xor_scramble", ctypes.c_void_p), ("xor_reorder", ctypes.c_void_p),
                ("shift_table", ctypes.c_void_p)]


class Integrand(ctypes.Structure):
    """Mirror of qmc_integrand."""
    _fields_ = [("kind", ctypes.c_uint32), ("d", ctypes.c_uint32), ("num_lobes", ctypes.c_uint32),
                ("pixel_seed", ctypes.c_uint32), ("params", ctypes.c_void_p), ("pixel_params", ctypes.c_void_p)]


class QMCError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_vp = ctypes.c_void_p
_st = ctypes.c_int

# name -> (restype, argtypes); every symbol the public header declares.
SIGNATURES = {
    "qmc_create": (_st, [ctypes.c_int, ctypes.POINTER(_vp)]),
    "qmc_destroy": (_st, [_vp]),
    "qmc_last_error": (ctypes.c_char_p, []),
    "qmc_version": (ctypes.c_char_p, []),
    "qmc_primitive_polynomials": (_st, [_u32, _vp]),
    "qmc_sobol_matrices": (_st, [_u32, _vp, _vp]),
    "qmc_map_u32_to_unifloat": (_st, [_vp, _vp, _vp, _vp, _u64]),
    "qmc_generate_sobol": (_st, [_vp, _vp, _vp, _u32, _u64, _u64, _vp, _vp, _u32, _vp, _vp, _u64]),
    "qmc_generate_lattice": (_st, [_vp, _vp, _vp, _u32, _u64, _u64, _vp, _u32, _vp, _vp, _u64]),
    "qmc_generate_halton": (_st, [_vp, _vp, _u32, _u64, _u64, _u32, _vp, _vp, _vp, _u64]),
    "qmc_sobol_matrices_wide": (_st, [_u32, _vp, _u32, _vp]),
    "qmc_generate_sobol64": (_st, [_vp, _vp, _vp, _u32, _u32, _u32, _u32, _u64, _u64, _vp, _vp, _u32, _vp, _vp,
                                   _u64]),
    "qmc_generate_lattice64": (_st, [_vp, _vp, _vp, _u32, _u32, _u32, _u64, _u64, _vp, _u32, _vp, _vp, _u64]),
    "qmc_workspace_size": (_st, [_vp, _vp, _vp, _u32, _u32, ctypes.c_int, ctypes.POINTER(ctypes.c_size_t)]),
    "qmc_integrate_pixels": (_st, [_vp, _vp, _vp, _vp, _u32, _u32, _vp, _u32, _u32, _vp, _vp, _vp,
                                   ctypes.c_size_t]),
    "qmc_integrate_pixels_backward": (_st, [_vp, _vp, _vp, _vp, _u32, _u32, _vp, _u32, _u32, _vp, _vp, _vp,
                                            ctypes.c_size_t]),
    "qmc_integrate_pixels_l2_step": (_st, [_vp, _vp, _vp, _vp, _u32, _u32, _vp, _vp, _vp, _vp, _vp, _vp,
                                           ctypes.c_size_t]),
    "qmc_integrate_pixels_l2_step_noalloc": (_st, [_vp, _vp, _vp, _vp, _u32, _u32, _vp, _vp, _vp, _vp, _vp]),
    "qmc_sample_offsets": (_st, [_vp, _vp, _vp, _u32, _vp, _vp, ctypes.c_size_t]),
    "qmc_generate_pixel_samples": (_st, [_vp, _vp, _vp, _u32, _u32, _u32, _vp, _vp, _vp, _u64, _vp,
                                         ctypes.c_size_t]),
    "qmc_integrate_progressive": (_st, [_vp, _vp, _vp, _vp, _u32, _u32, _vp, _u32, _u32, _vp, _vp, _vp,
                                        ctypes.c_size_t, ctypes.c_int]),
    "qmc_autotune_generate": (_st, [_vp, _vp, _u32, _vp, _u32, _u64, _vp, _vp, _vp, _vp, _vp, ctypes.c_size_t]),
    "qmc_autotune_integrate": (_st, [_vp, _vp, _vp, _vp, _u32, _u32, _vp, _u32, _u32, ctypes.c_int, _vp, _vp,
                                     _vp, ctypes.c_size_t, _vp, ctypes.c_size_t]),
    "qmc_tune_save": (_st, [_vp, ctypes.c_char_p]),
    "qmc_tune_load": (_st, [_vp, ctypes.c_char_p]),
}

_lib = None


def load():
    """The loaded library (cached).  Raises if libqmc.so has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libqmc.so not found at %s; build it with "
                          "`python -m paper_2307_15584_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status):
    if status != QMC_OK:
        msg = load().qmc_last_error()
        raise QMCError(status, msg.decode() if msg else "")
