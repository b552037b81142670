"""Python binding of libqmc (MI355X / gfx950 quasi-Monte Carlo sampling and integration).

Thin argument marshalling over the C ABI declared in include/qmc.h: every function here
has the name of the C entry point it calls, takes torch tensors for device buffers and
passes their pointers and the current torch stream.  All computation happens in the HIP
kernels of libqmc.so; torch only provides device memory and streams.

u32 data lives in torch.int32 tensors (same bits); use `to_u32(t)` to view it on the host.
"""

import ctypes

import numpy as np

from ._lib import (  # noqa: F401
    QMC_F_GENZ,
    QMC_F_LOBES,
    QMC_HALTON_FAURE,
    QMC_HALTON_IDENTITY,
    QMC_HALTON_LINEAR,
    QMC_LATTICE_BACKWARD,
    QMC_LATTICE_INSTANCES4,
    QMC_MAX_DEGREE,
    QMC_MAX_DIMS,
    QMC_PIXEL_HILBERT_SHIFT,
    QMC_PIXEL_TABLE_SHIFT,
    QMC_PIXEL_NUS,
    QMC_PIXEL_RANDOM_GENERATOR,
    QMC_PIXEL_SHIFT,
    QMC_POINT_MAJOR,
    QMC_SAMPLER_LATTICE,
    QMC_SAMPLER_POINTS,
    QMC_SAMPLER_SOBOL,
    QMC_SAMPLER_XOR_TABLE,
    QMC_XOR_TABLE_CELLS,
    QMC_SHIFT_XOR,
    QMC_STATIC_SCRATCH_BYTES,
    Integrand,
    QMCError,
    Sampler,
    check,
    load,
)

_contexts = {}


def _torch():
    import torch

    return torch


def context(device=None):
    """The library context of a CUDA/HIP device (created on first use, kept for the process)."""
    torch = _torch()
    if device is None:
        device = torch.cuda.current_device()
    if isinstance(device, torch.device):
        device = device.index if device.index is not None else torch.cuda.current_device()
    if device not in _contexts:
        h = ctypes.c_void_p()
        check(load().qmc_create(int(device), ctypes.byref(h)))
        _contexts[device] = h
    return _contexts[device]


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def _dev_ptr(t, name, dtype=None):
    """Device pointer of a contiguous GPU tensor (or None)."""
    if t is None:
        return None
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if dtype is not None and t.dtype not in dtype:
        raise TypeError("%s has dtype %s, expected one of %s" % (name, t.dtype, dtype))
    return ctypes.c_void_p(t.data_ptr())


def _device_of(*ts):
    for t in ts:
        if t is not None:
            return t.device
    return None


def to_u32(t):
    """Host numpy uint32 view of a tensor holding u32 bit patterns."""
    return t.detach().cpu().contiguous().numpy().view(np.uint32)


def from_u32(a, device="cuda"):
    """Device int32 tensor holding the bits of a uint32 numpy array."""
    torch = _torch()
    a = np.ascontiguousarray(np.asarray(a, dtype=np.uint32))
    return torch.from_numpy(a.view(np.int32).copy()).to(device)


def _u32_types():
    torch = _torch()
    return (torch.int32, torch.uint32) if hasattr(torch, "uint32") else (torch.int32,)


# ------------------------------------------------------------------ setup (host) ----

def qmc_primitive_polynomials(count):
    """The first `count` primitive polynomials over F_2 as uint32 codes (host numpy)."""
    out = np.zeros(max(count, 1), dtype=np.uint32)
    check(load().qmc_primitive_polynomials(count, out.ctypes.data_as(ctypes.c_void_p)))
    return out[:count]


def qmc_sobol_matrices(s, direction_init):
    """Sobol' generator matrices uint32 [s][32] (host numpy) from direction_init [s][16]."""
    di = np.ascontiguousarray(np.asarray(direction_init, dtype=np.uint32))
    if di.shape != (s, QMC_MAX_DEGREE):
        raise ValueError("direction_init must have shape (%d, %d)" % (s, QMC_MAX_DEGREE))
    out = np.zeros((s, 32), dtype=np.uint32)
    check(load().qmc_sobol_matrices(s, di.ctypes.data_as(ctypes.c_void_p), out.ctypes.data_as(ctypes.c_void_p)))
    return out


def qmc_sobol_matrices_wide(s, direction_init, columns):
    """Sobol' generator matrices uint32 [s][columns] (host numpy) for indices of up to
    `columns` <= 64 bits; the first 32 columns equal qmc_sobol_matrices'."""
    di = np.ascontiguousarray(np.asarray(direction_init, dtype=np.uint32))
    if di.shape != (s, QMC_MAX_DEGREE):
        raise ValueError("direction_init must have shape (%d, %d)" % (s, QMC_MAX_DEGREE))
    out = np.zeros((s, max(int(columns), 1)), dtype=np.uint32)
    check(load().qmc_sobol_matrices_wide(s, di.ctypes.data_as(ctypes.c_void_p), columns,
                                         out.ctypes.data_as(ctypes.c_void_p)))
    return out


# ------------------------------------------------------------- generation (device) ----

def qmc_map_u32_to_unifloat(inp, out=None):
    """out = map_u32_to_unifloat(inp) elementwise on the GPU; returns out (float32)."""
    torch = _torch()
    if out is None:
        out = torch.empty(inp.shape, dtype=torch.float32, device=inp.device)
    pi = _dev_ptr(inp, "inp", _u32_types())
    po = _dev_ptr(out, "out", (torch.float32,))
    if out.numel() != inp.numel():
        raise ValueError("out must have as many elements as inp")
    check(load().qmc_map_u32_to_unifloat(context(inp.device), _stream(), pi, po, inp.numel()))
    return out


def _check_len(t, s, name):
    if t is not None and t.numel() < s:
        raise ValueError("%s needs at least %d entries" % (name, s))


def _outputs(s, n, ld, out_u32, out_f32, want_u32, want_f32, device, point_major=False):
    """Output tensors: [s][ld] (dimension-major) or [n][ld] (point-major, ld >= s)."""
    torch = _torch()
    ld = (s if point_major else n) if ld is None else ld
    shape = (n, ld) if point_major else (s, ld)
    if out_u32 is None and want_u32:
        out_u32 = torch.empty(shape, dtype=torch.int32, device=device)
    if out_f32 is None and want_f32:
        out_f32 = torch.empty(shape, dtype=torch.float32, device=device)
    need = (n - 1) * ld + s if point_major else (s - 1) * ld + n
    for t, name in ((out_u32, "out_u32"), (out_f32, "out_f32")):
        if t is not None and t.numel() < need:
            raise ValueError("%s is too small for s=%d, ld=%d, n=%d" % (name, s, ld, n))
    return ld, out_u32, out_f32


def qmc_generate_sobol(matrices, first, n, nus_seeds=None, shifts=None, flags=0, out_u32=None, out_f32=None,
                       ld=None, want_u32=True, want_f32=True):
    """Points i in [first, first+n) of the digital sequence with device matrices [s][32].

    Returns (u32 int32 tensor, float32 tensor), each [s][ld] ([n][ld] with QMC_POINT_MAJOR) or None.
    """
    torch = _torch()
    s = matrices.shape[0]
    if matrices.numel() != s * 32:
        raise ValueError("matrices must have shape [s][32]")
    _check_len(nus_seeds, s, "nus_seeds")
    _check_len(shifts, s, "shifts")
    ld, out_u32, out_f32 = _outputs(s, n, ld, out_u32, out_f32, want_u32, want_f32, matrices.device,
                                    bool(flags & QMC_POINT_MAJOR))
    st = load().qmc_generate_sobol(
        context(matrices.device), _stream(), _dev_ptr(matrices, "matrices", _u32_types()), s, first, n,
        _dev_ptr(nus_seeds, "nus_seeds", _u32_types()), _dev_ptr(shifts, "shifts", _u32_types()), flags,
        _dev_ptr(out_u32, "out_u32", _u32_types()), _dev_ptr(out_f32, "out_f32", (torch.float32,)), ld)
    check(st)
    return out_u32, out_f32


def qmc_generate_lattice(generator, first, n, shifts=None, flags=0, out_u32=None, out_f32=None, ld=None,
                         want_u32=True, want_f32=True):
    """Points i in [first, first+n) of the rank-1 lattice sequence with device generator [s]."""
    torch = _torch()
    s = generator.shape[0]
    if generator.dim() != 1:
        raise ValueError("generator must be a vector [s]")
    _check_len(shifts, s, "shifts")
    ld, out_u32, out_f32 = _outputs(s, n, ld, out_u32, out_f32, want_u32, want_f32, generator.device,
                                    bool(flags & QMC_POINT_MAJOR))
    st = load().qmc_generate_lattice(
        context(generator.device), _stream(), _dev_ptr(generator, "generator", _u32_types()), s, first, n,
        _dev_ptr(shifts, "shifts", _u32_types()), flags,
        _dev_ptr(out_u32, "out_u32", _u32_types()), _dev_ptr(out_f32, "out_f32", (torch.float32,)), ld)
    check(st)
    return out_u32, out_f32


def qmc_generate_sobol64(matrices, first, n, log2_parts=0, part=0, nus_seeds=None, shifts=None, flags=0,
                         out_u32=None, out_f32=None, ld=None, want_u32=True, want_f32=True):
    """Points m in [first, first+n) of part `part` of 2^log2_parts (global index
    m 2^log2_parts + rev(part)) of the digital sequence with device matrices [s][columns],
    64-bit indices.  Returns (u32 int32 tensor [s][ld] or None, float32 tensor or None)."""
    torch = _torch()
    if matrices.dim() != 2:
        raise ValueError("matrices must have shape [s][columns]")
    s, columns = matrices.shape
    _check_len(nus_seeds, s, "nus_seeds")
    _check_len(shifts, s, "shifts")
    ld, out_u32, out_f32 = _outputs(s, n, ld, out_u32, out_f32, want_u32, want_f32, matrices.device)
    st = load().qmc_generate_sobol64(
        context(matrices.device), _stream(), _dev_ptr(matrices, "matrices", _u32_types()), columns, s, log2_parts,
        part, first, n, _dev_ptr(nus_seeds, "nus_seeds", _u32_types()), _dev_ptr(shifts, "shifts", _u32_types()),
        flags, _dev_ptr(out_u32, "out_u32", _u32_types()), _dev_ptr(out_f32, "out_f32", (torch.float32,)), ld)
    check(st)
    return out_u32, out_f32


def qmc_generate_lattice64(generator, first, n, log2_parts=0, part=0, shifts=None, flags=0, out_u32=None,
                           out_f32=None, ld=None, want_u32=True, want_f32=True):
    """Points m in [first, first+n) of part `part` of 2^log2_parts of the rank-1 lattice
    sequence with device generator [s], 64-bit indices."""
    torch = _torch()
    if generator.dim() != 1:
        raise ValueError("generator must be a vector [s]")
    s = generator.shape[0]
    _check_len(shifts, s, "shifts")
    ld, out_u32, out_f32 = _outputs(s, n, ld, out_u32, out_f32, want_u32, want_f32, generator.device)
    st = load().qmc_generate_lattice64(
        context(generator.device), _stream(), _dev_ptr(generator, "generator", _u32_types()), s, log2_parts, part,
        first, n, _dev_ptr(shifts, "shifts", _u32_types()), flags,
        _dev_ptr(out_u32, "out_u32", _u32_types()), _dev_ptr(out_f32, "out_f32", (torch.float32,)), ld)
    check(st)
    return out_u32, out_f32


def qmc_generate_halton(s, first, n, mode=0, factors=None, out_u32=None, out_f32=None, ld=None, want_u32=True,
                        want_f32=True, device="cuda"):
    """Points i in [first, first+n) of the Halton sequence in s dimensions (bases: the first s
    primes), with QMC_HALTON_IDENTITY / _FAURE / _LINEAR digit permutations; factors: device
    u32 [s] for _LINEAR.  Returns (u32 int32 tensor [s][ld] or None, float32 tensor or None)."""
    torch = _torch()
    _check_len(factors, s, "factors")
    dev = factors.device if factors is not None else torch.device(device)
    ld, out_u32, out_f32 = _outputs(s, n, ld, out_u32, out_f32, want_u32, want_f32, dev)
    st = load().qmc_generate_halton(
        context(dev), _stream(), s, first, n, mode, _dev_ptr(factors, "factors", _u32_types()),
        _dev_ptr(out_u32, "out_u32", _u32_types()), _dev_ptr(out_f32, "out_f32", (torch.float32,)), ld)
    check(st)
    return out_u32, out_f32


# -------------------------------------------------------- per-pixel integration ----

class PixelSampler:
    """A qmc_sampler plus the device tensors it points to (kept alive with it)."""

    def __init__(self, kind, table, seed=0, flags=0, points_ld=0, offsets=None, s=None, xor_scramble=None,
                 xor_reorder=None, shift_table=None):
        self.table = table
        self.offsets = offsets
        self.xor_scramble, self.xor_reorder, self.shift_table = xor_scramble, xor_reorder, shift_table
        self.kind = kind
        self.seed = seed
        self.flags = flags
        if s is None:
            s = table.shape[0]
        self.s = s
        torch = _torch()
        opt = lambda t, name, types=None: _dev_ptr(t, name, types).value if t is not None else None
        u32 = _u32_types()
        tab_types = (torch.float32,) if kind == QMC_SAMPLER_POINTS else u32
        self.c = Sampler(kind, s, _dev_ptr(table, "table", tab_types).value, points_ld, opt(offsets, "offsets"),
                         seed & 0xFFFFFFFF, flags, opt(xor_scramble, "xor_scramble", u32),
                         opt(xor_reorder, "xor_reorder", u32), opt(shift_table, "shift_table", u32))

    @staticmethod
    def _table_flags(flags, shift_table):
        if shift_table is None:
            return flags
        if tuple(shift_table.shape) != (2, QMC_XOR_TABLE_CELLS):
            raise ValueError("shift_table must be [2][16384]")
        return flags | QMC_PIXEL_SHIFT | QMC_PIXEL_TABLE_SHIFT

    @classmethod
    def sobol(cls, matrices, seed, flags=QMC_PIXEL_NUS | QMC_PIXEL_SHIFT, shift_table=None):
        """shift_table: optional u32 [2][16384] per-pixel rotations (Sec. 2.6.1) replacing the hashed ones."""
        if matrices.numel() != matrices.shape[0] * 32:
            raise ValueError("matrices must have shape [s][32]")
        return cls(QMC_SAMPLER_SOBOL, matrices, seed, cls._table_flags(flags, shift_table), shift_table=shift_table)

    @classmethod
    def lattice(cls, generator, seed, flags=QMC_PIXEL_SHIFT, shift_table=None):
        return cls(QMC_SAMPLER_LATTICE, generator, seed, cls._table_flags(flags, shift_table),
                   shift_table=shift_table)

    @classmethod
    def xor_table(cls, points, scramble, reorder):
        """Stored points u32 [s][N] (N a power of two), digit scrambles u32 [s][16384] and index
        reorderings u32 [16384] of the 128 x 128 pixel tables (Sec. 2.6.1)."""
        s, n = points.shape
        if n == 0 or n & (n - 1) or n > 1 << 32:
            raise ValueError("the number of stored points must be a power of two <= 2^32")
        if tuple(scramble.shape) != (s, QMC_XOR_TABLE_CELLS) or reorder.numel() != QMC_XOR_TABLE_CELLS:
            raise ValueError("scramble must be [s][16384] and reorder [16384]")
        return cls(QMC_SAMPLER_XOR_TABLE, points, 0, 0, points_ld=n, s=s, xor_scramble=scramble, xor_reorder=reorder)

    @classmethod
    def points(cls, samples, offsets):
        """Materialised samples [d][ld] float32 with per-pixel offsets (int64 [P+1]); sample i of
        pixel p is column offsets[p] + i, so offsets[P] must not exceed ld."""
        torch = _torch()
        if samples.dim() != 2 or samples.dtype != torch.float32:
            raise TypeError("samples must be a float32 tensor [d][ld]")
        if offsets.dim() != 1 or offsets.dtype != torch.int64:
            raise TypeError("offsets must be an int64 vector [P+1]")
        return cls(QMC_SAMPLER_POINTS, samples, 0, 0, points_ld=samples.shape[1], offsets=offsets,
                   s=samples.shape[0])


class PixelIntegrand:
    """A qmc_integrand plus its device tensors."""

    def __init__(self, kind, d, params=None, pixel_params=None, num_lobes=0, pixel_seed=0):
        self.params = params
        self.pixel_params = pixel_params
        self.kind, self.d, self.num_lobes, self.pixel_seed = kind, d, num_lobes, pixel_seed
        torch = _torch()
        self.c = Integrand(kind, d, num_lobes, pixel_seed & 0xFFFFFFFF,
                           _dev_ptr(params, "params", (torch.float32,)).value if params is not None else None,
                           _dev_ptr(pixel_params, "pixel_params", (torch.float32,)).value
                           if pixel_params is not None else None)

    @classmethod
    def genz(cls, pixel_params):
        return cls(QMC_F_GENZ, 8, pixel_params=pixel_params)

    @classmethod
    def lobes(cls, params, num_lobes, d, pixel_seed):
        if params.numel() != num_lobes * (2 * d + 1):
            raise ValueError("params must have L*(2d+1) entries")
        return cls(QMC_F_LOBES, d, params=params, num_lobes=num_lobes, pixel_seed=pixel_seed)

    def with_params(self, params):
        return PixelIntegrand(self.kind, self.d, params, self.pixel_params, self.num_lobes, self.pixel_seed)


def qmc_workspace_size(sampler, integrand, width, height, backward=False):
    """Workspace bytes: backward False/0 forward, True/1 adjoint, 2 fused L2 step."""
    n = ctypes.c_size_t()
    check(load().qmc_workspace_size(context(), ctypes.byref(sampler.c), ctypes.byref(integrand.c), width, height,
                                    int(backward), ctypes.byref(n)))
    return n.value


def _workspace(nbytes, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def _check_counts(counts, P, sampler=None):
    if counts.numel() != P:
        raise ValueError("counts must have width*height entries")
    if sampler is not None and sampler.kind == QMC_SAMPLER_POINTS and sampler.offsets.numel() != P + 1:
        raise ValueError("the POINTS sampler's offsets must have width*height + 1 entries")


def qmc_integrate_pixels(sampler, integrand, width, height, counts, sample_begin=0, sample_end=0xFFFFFFFF,
                         sums=None, means=None, workspace=None):
    """Per-pixel estimates; returns means (allocated when neither sums nor means is given)."""
    torch = _torch()
    P = width * height
    _check_counts(counts, P, sampler)
    if sums is None and means is None:
        means = torch.empty(P, dtype=torch.float32, device=counts.device)
    for t, nm in ((sums, "sums"), (means, "means")):
        if t is not None and t.numel() != P:
            raise ValueError("%s must have width*height entries" % nm)
    if workspace is None:
        workspace = _workspace(qmc_workspace_size(sampler, integrand, width, height, False), counts.device)
    check(load().qmc_integrate_pixels(
        context(counts.device), _stream(), ctypes.byref(sampler.c), ctypes.byref(integrand.c), width, height,
        _dev_ptr(counts, "counts", _u32_types()), sample_begin, sample_end,
        _dev_ptr(sums, "sums", (torch.float32,)), _dev_ptr(means, "means", (torch.float32,)),
        _dev_ptr(workspace, "workspace"), workspace.numel()))
    return means if means is not None else sums


def qmc_integrate_pixels_backward(sampler, integrand, width, height, counts, grad_means, grad_params=None,
                                  sample_begin=0, sample_end=0xFFFFFFFF, workspace=None):
    """Adds dL/dtheta into grad_params (zeros if not given); returns grad_params."""
    torch = _torch()
    P = width * height
    _check_counts(counts, P, sampler)
    if grad_means.numel() != P:
        raise ValueError("grad_means must have width*height entries")
    if grad_params is None:
        grad_params = torch.zeros(integrand.params.numel(), dtype=torch.float32, device=counts.device)
    if workspace is None:
        workspace = _workspace(qmc_workspace_size(sampler, integrand, width, height, True), counts.device)
    check(load().qmc_integrate_pixels_backward(
        context(counts.device), _stream(), ctypes.byref(sampler.c), ctypes.byref(integrand.c), width, height,
        _dev_ptr(counts, "counts", _u32_types()), sample_begin, sample_end,
        _dev_ptr(grad_means, "grad_means", (torch.float32,)), _dev_ptr(grad_params, "grad_params", (torch.float32,)),
        _dev_ptr(workspace, "workspace"), workspace.numel()))
    return grad_params


def qmc_integrate_pixels_l2_step(sampler, integrand, width, height, counts, target, means=None, loss=None,
                                 grad_params=None, workspace=None):
    """Fused forward + L2-loss gradient + adjoint.  Returns (means, loss[1], grad_params);
    loss and grad_params are added into (zeros when not given)."""
    torch = _torch()
    P = width * height
    _check_counts(counts, P, sampler)
    if target.numel() != P:
        raise ValueError("target must have width*height entries")
    if means is None:
        means = torch.empty(P, dtype=torch.float32, device=counts.device)
    if loss is None:
        loss = torch.zeros(1, dtype=torch.float32, device=counts.device)
    if grad_params is None:
        grad_params = torch.zeros(integrand.params.numel(), dtype=torch.float32, device=counts.device)
    if workspace is None:
        workspace = _workspace(qmc_workspace_size(sampler, integrand, width, height, 2), counts.device)
    check(load().qmc_integrate_pixels_l2_step(
        context(counts.device), _stream(), ctypes.byref(sampler.c), ctypes.byref(integrand.c), width, height,
        _dev_ptr(counts, "counts", _u32_types()), _dev_ptr(target, "target", (torch.float32,)),
        _dev_ptr(means, "means", (torch.float32,)), _dev_ptr(loss, "loss", (torch.float32,)),
        _dev_ptr(grad_params, "grad_params", (torch.float32,)), _dev_ptr(workspace, "workspace"), workspace.numel()))
    return means, loss, grad_params


def qmc_integrate_pixels_l2_step_noalloc(sampler, integrand, width, height, counts, target, means, loss,
                                         grad_params):
    """The fused training step of qmc_integrate_pixels_l2_step without a workspace: the library's
    static scratch on the device holds its work counter and accumulator, and nothing is allocated
    (means, loss and grad_params are required; loss and grad_params are added into).  Calls that
    overlap on one GPU share that scratch and must be ordered by the caller."""
    torch = _torch()
    P = width * height
    _check_counts(counts, P, sampler)
    if target.numel() != P or means.numel() != P:
        raise ValueError("target and means must have width*height entries")
    check(load().qmc_integrate_pixels_l2_step_noalloc(
        context(counts.device), _stream(), ctypes.byref(sampler.c), ctypes.byref(integrand.c), width, height,
        _dev_ptr(counts, "counts", _u32_types()), _dev_ptr(target, "target", (torch.float32,)),
        _dev_ptr(means, "means", (torch.float32,)), _dev_ptr(loss, "loss", (torch.float32,)),
        _dev_ptr(grad_params, "grad_params", (torch.float32,))))
    return means, loss, grad_params


def qmc_sample_offsets(counts):
    """int64 [P+1] exclusive prefix sums of counts (computed on the GPU)."""
    torch = _torch()
    P = counts.numel()
    offsets = torch.empty(P + 1, dtype=torch.int64, device=counts.device)
    ws = _workspace(8 * (P // 1024 + 2), counts.device)
    check(load().qmc_sample_offsets(context(counts.device), _stream(), _dev_ptr(counts, "counts", _u32_types()), P,
                                    _dev_ptr(offsets, "offsets"), _dev_ptr(ws, "workspace"), ws.numel()))
    return offsets


def qmc_generate_pixel_samples(sampler, d, width, height, counts, offsets, total, out=None):
    """Materialised samples float32 [d][total] (the plain path's generation step).

    offsets: int64 [P+1], the exclusive prefix sums of counts (qmc_sample_offsets), whose last
    entry is `total`; out: float32 [>= d][>= total].  The kernel writes column offsets[p] + i
    for sample i of pixel p, so these shapes bound every store."""
    torch = _torch()
    P = width * height
    _check_counts(counts, P)
    if not isinstance(offsets, torch.Tensor) or offsets.dtype != torch.int64 or offsets.numel() != P + 1:
        raise TypeError("offsets must be an int64 tensor of width*height + 1 entries")
    if out is None:
        out = torch.empty((d, max(int(total), 1)), dtype=torch.float32, device=counts.device)
    if out.dtype != torch.float32 or out.dim() != 2:
        raise TypeError("out must be a float32 tensor [d][ld]")
    if out.shape[0] < d or out.shape[1] < total:
        raise ValueError("out has shape %s; [>= %d][>= %d] needed" % (tuple(out.shape), d, total))
    ws = _workspace(1024, counts.device)
    check(load().qmc_generate_pixel_samples(
        context(counts.device), _stream(), ctypes.byref(sampler.c), d, width, height,
        _dev_ptr(counts, "counts", _u32_types()), _dev_ptr(offsets, "offsets"), _dev_ptr(out, "out"),
        out.shape[1], _dev_ptr(ws, "workspace"), ws.numel()))
    return out


def qmc_integrate_progressive(sampler, integrand, width, height, counts, passes, spp_per_pass, sums, means=None,
                              workspace=None, use_graph=True):
    """passes x spp_per_pass windows added into sums (graph-captured and replayed when use_graph)."""
    torch = _torch()
    P = width * height
    _check_counts(counts, P, sampler)
    if workspace is None:
        workspace = _workspace(qmc_workspace_size(sampler, integrand, width, height, False), counts.device)
    check(load().qmc_integrate_progressive(
        context(counts.device), _stream(), ctypes.byref(sampler.c), ctypes.byref(integrand.c), width, height,
        _dev_ptr(counts, "counts", _u32_types()), passes, spp_per_pass, _dev_ptr(sums, "sums", (torch.float32,)),
        _dev_ptr(means, "means", (torch.float32,)), _dev_ptr(workspace, "workspace"), workspace.numel(),
        1 if use_graph else 0))
    return sums


def qmc_autotune_generate(kind, table, n, nus_seeds=None, shifts=None, scratch_u32=None, scratch_f32=None):
    """Tunes the materialising kernels of one sequence kind; returns the per-candidate report."""
    torch = _torch()
    s = table.shape[0]
    if scratch_u32 is None and scratch_f32 is None:
        scratch_u32 = torch.empty((s, n), dtype=torch.int32, device=table.device)
        scratch_f32 = torch.empty((s, n), dtype=torch.float32, device=table.device)
    rep = ctypes.create_string_buffer(8192)
    check(load().qmc_autotune_generate(
        context(table.device), _stream(), kind, _dev_ptr(table, "table"), s, n, _dev_ptr(nus_seeds, "nus_seeds"),
        _dev_ptr(shifts, "shifts"), _dev_ptr(scratch_u32, "scratch_u32"), _dev_ptr(scratch_f32, "scratch_f32"),
        rep, len(rep)))
    return rep.value.decode()


def qmc_autotune_integrate(sampler, integrand, width, height, counts, sample_begin=0, sample_end=0xFFFFFFFF,
                           backward=False, grad_means=None):
    """Tunes the integration launch shape for this problem; returns the per-candidate report."""
    torch = _torch()
    P = width * height
    n = integrand.params.numel() if backward else P
    scratch = torch.zeros(n, dtype=torch.float32, device=counts.device)
    ws = _workspace(qmc_workspace_size(sampler, integrand, width, height, backward), counts.device)
    rep = ctypes.create_string_buffer(8192)
    check(load().qmc_autotune_integrate(
        context(counts.device), _stream(), ctypes.byref(sampler.c), ctypes.byref(integrand.c), width, height,
        _dev_ptr(counts, "counts", _u32_types()), sample_begin, sample_end, 1 if backward else 0,
        _dev_ptr(grad_means, "grad_means"), _dev_ptr(scratch, "scratch"), _dev_ptr(ws, "workspace"), ws.numel(),
        rep, len(rep)))
    return rep.value.decode()


def qmc_tune_save(path):
    check(load().qmc_tune_save(context(), path.encode()))


def qmc_tune_load(path):
    check(load().qmc_tune_load(context(), path.encode()))


from .autograd import QMCIntegrate, integrate  # noqa: E402,F401
