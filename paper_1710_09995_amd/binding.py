"""ctypes binding over libcfd.so (include/cfd.h).

Argument marshalling only: torch owns every device buffer (state arena,
workspace, node upload, residual, history) and supplies the HIP stream; every
step of the computation runs in the library's HIP kernels.  There is no CPU
fallback: if the shared library cannot be loaded the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import List, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.environ.get("CFD_LIB", os.path.join(HERE, "libcfd.so"))
NG = 2

CFD_OK = 0
STATUS = {0: "CFD_OK", -1: "CFD_EINVAL", -2: "CFD_ENOMEM", -3: "CFD_EHIP", -4: "CFD_ENONFINITE",
          -5: "CFD_ESTATE", -6: "CFD_EUNSUPPORTED", -7: "CFD_EINTERNAL"}
CFD_NORMS_HOST = 1


class Dims(C.Structure):
    _fields_ = [("ni", C.c_int32), ("nj", C.c_int32), ("nk", C.c_int32)]


class ConnS(C.Structure):
    _fields_ = [("blk", C.c_int32), ("face", C.c_int32), ("nbr", C.c_int32), ("nbr_face", C.c_int32),
                ("lo", C.c_int32 * 2), ("hi", C.c_int32 * 2), ("nbr_lo", C.c_int32 * 2),
                ("shift", C.c_double * 3)]


class BCS(C.Structure):
    _fields_ = [("blk", C.c_int32), ("face", C.c_int32), ("kind", C.c_int32),
                ("lo", C.c_int32 * 2), ("hi", C.c_int32 * 2), ("pad", C.c_int32), ("mach", C.c_double)]


class PieceS(C.Structure):
    _fields_ = [("parent", C.c_int32), ("lo", C.c_int32 * 3), ("n", C.c_int32 * 3)]


class ParamsS(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("gamma", "prandtl", "mach", "alpha", "beta", "reynolds",
                                           "sutherland", "cfl", "entropy_fix", "limiter_eps")] + \
               [(n, C.c_int32) for n in ("viscous", "flux_fp32", "local_dt", "ghost_layers")]


class Tuning(C.Structure):
    _fields_ = [("kernel", C.c_int32), ("tile_j", C.c_int32), ("tile_k", C.c_int32),
                ("use_graph", C.c_int32), ("order", C.c_int32)]


class WcnsClosure(C.Structure):
    _fields_ = [("owner", C.c_int32), ("ghost_lo", C.c_int32), ("ghost_hi", C.c_int32), ("bounded", C.c_int32),
                ("kind", C.c_int32 * 2), ("uinf", C.c_double * 3)]


class MlpDesc(C.Structure):
    _fields_ = [("d_in", C.c_int32), ("d_hidden", C.c_int32), ("n_hidden", C.c_int32), ("d_out", C.c_int32),
                ("activation", C.c_int32)]


EXPORTS = ["cfd_layout", "cfd_workspace_size", "cfd_create_blocks", "cfd_destroy", "cfd_set_tuning",
           "cfd_get_tuning", "cfd_fill_ghosts", "cfd_residual", "cfd_step", "cfd_implicit_work_size",
           "cfd_step_implicit", "cfd_mg_work_size", "cfd_mg_cycles", "cfd_norms",
           "cfd_time_step", "cfd_copy_metrics", "cfd_set_profiling", "cfd_profile_read",
           "cfd_mlp_sizes", "cfd_mlp_forward", "cfd_mlp_mse", "cfd_mlp_backward", "cfd_mlp_adam",
           "cfd_mlp_to_bf16", "cfd_mlp_features", "cfd_mlp_targets", "cfd_mlp_to_state",
           "cfd_split_plan", "cfd_split_tables", "cfd_regroup", "cfd_staggered_diff6", "cfd_wcns5_edges",
           "cfd_wcns5_euler_work_bytes", "cfd_wcns5_euler_residual_periodic",
           "cfd_wcns5_euler_residual_periodic_noalloc", "cfd_wcns5_euler_step_work_bytes",
           "cfd_wcns5_euler_steps_periodic", "cfd_c4_viscous_work_bytes", "cfd_c4_viscous_add_periodic",
           "cfd_wcns5_metrics_periodic", "cfd_wcns5_euler_residual_curv_periodic",
           "cfd_wcns5_euler_steps_curv_periodic", "cfd_c4_viscous_curv_work_bytes",
           "cfd_c4_viscous_add_curv_periodic", "cfd_wcns5_time_step_curv_periodic", "cfd_wcns5_metrics_ext",
           "cfd_wcns5_euler_blocks_work_bytes", "cfd_wcns5_euler_residual_blocks", "cfd_c4_viscous_blocks_work_bytes",
           "cfd_c4_viscous_add_blocks", "cfd_wcns5_ns_step_work_bytes", "cfd_wcns5_ns_steps_curv_periodic",
           "cfd_wcns5_implicit_step_work_bytes", "cfd_wcns5_implicit_steps_curv_periodic",
           "cfd_wcns5_implicit_blocks_work_bytes", "cfd_wcns5_implicit_steps_blocks", "cfd_wcns5_ns_blocks_work_bytes",
           "cfd_wcns5_ns_steps_blocks", "cfd_wcns5_extend_vertices", "cfd_wcns5_extend_vertices_mask",
           "cfd_wcns5_fill_ghost_blocks",
           "cfd_wcns5_steps_blocks_closed",
           "cfd_status_string", "cfd_last_error"]

_lib = None


def lib(build_if_missing: bool = True):
    """Load libcfd.so (building it first only if no built library exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIBPATH):
        if not build_if_missing:
            raise RuntimeError(f"{LIBPATH} is missing; run python -m paper_1710_09995_amd.build")
        from . import build as _b
        _b.build()
    L = C.CDLL(LIBPATH)
    vp, i32, i64p = C.c_void_p, C.c_int32, C.POINTER(C.c_int64)
    L.cfd_layout.argtypes = [i32, C.POINTER(Dims), i32, i64p, i64p, i64p]
    L.cfd_workspace_size.argtypes = [C.POINTER(ParamsS), i32, C.POINTER(Dims), C.POINTER(C.c_size_t)]
    L.cfd_create_blocks.argtypes = [C.POINTER(ParamsS), i32, C.POINTER(Dims), C.POINTER(vp), i32,
                                    C.POINTER(ConnS), i32, C.POINTER(BCS), vp, C.c_size_t, vp,
                                    C.POINTER(vp)]
    L.cfd_destroy.argtypes = [vp]
    L.cfd_set_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.cfd_get_tuning.argtypes = [vp, C.POINTER(Tuning)]
    L.cfd_fill_ghosts.argtypes = [vp, vp, vp]
    L.cfd_residual.argtypes = [vp, vp, vp, vp]
    L.cfd_step.argtypes = [vp, vp, i32, vp, vp]
    L.cfd_implicit_work_size.argtypes = [vp, C.POINTER(C.c_size_t)]
    L.cfd_step_implicit.argtypes = [vp, vp, i32, i32, C.c_double, vp, C.c_size_t, vp, vp]
    L.cfd_norms.argtypes = [vp, vp, vp, vp, i32, vp]
    L.cfd_time_step.argtypes = [vp, vp, vp, vp]
    L.cfd_copy_metrics.argtypes = [vp, i32, vp, vp]
    L.cfd_set_profiling.argtypes = [vp, i32]
    L.cfd_profile_read.argtypes = [vp, C.POINTER(C.c_double)]
    dp = C.POINTER(MlpDesc)
    L.cfd_mlp_sizes.argtypes = [dp, C.c_int64, i64p, i64p, C.POINTER(C.c_size_t)]
    L.cfd_mlp_forward.argtypes = [dp, vp, vp, vp, C.c_int64, vp, vp, vp]
    L.cfd_mlp_mse.argtypes = [dp, vp, vp, vp, C.c_int64, vp, vp, vp, C.c_size_t, vp]
    L.cfd_mlp_backward.argtypes = [dp, vp, vp, vp, C.c_int64, vp, vp, C.c_size_t, vp]
    L.cfd_mlp_adam.argtypes = [dp, vp, vp, vp, vp, vp, C.c_float, C.c_float, C.c_float, C.c_float, i32, vp]
    L.cfd_mlp_to_bf16.argtypes = [dp, vp, vp, vp]
    L.cfd_mlp_features.argtypes = [vp, vp, vp, vp]
    L.cfd_mlp_targets.argtypes = [vp, vp, vp, vp, vp]
    L.cfd_mlp_to_state.argtypes = [vp, vp, vp, vp, vp]
    i32p = C.POINTER(C.c_int32)
    L.cfd_split_plan.argtypes = [i32, C.POINTER(Dims), C.c_int64, i32, i32p, C.POINTER(PieceS), i32, i32p]
    L.cfd_split_tables.argtypes = [i32, C.POINTER(Dims), C.POINTER(ConnS), i32, C.POINTER(BCS), i32,
                                   C.POINTER(PieceS), i32, C.POINTER(ConnS), i32, i32p, C.POINTER(BCS), i32, i32p]
    L.cfd_regroup.argtypes = [i32, i64p, i32, C.POINTER(C.c_double), i32p, i64p]
    L.cfd_staggered_diff6.argtypes = [vp, vp, i32p, i32, i32, C.c_double, vp]
    L.cfd_wcns5_edges.argtypes = [vp, vp, vp, i32p, i32, i32, C.c_double, vp]
    L.cfd_wcns5_euler_work_bytes.argtypes = [i32p, C.POINTER(C.c_size_t)]
    L.cfd_wcns5_euler_residual_periodic.argtypes = [vp, vp, vp, C.c_size_t, i32p, C.POINTER(C.c_double), C.c_double,
                                                    C.c_double, C.c_double, vp]
    L.cfd_wcns5_euler_residual_periodic_noalloc.argtypes = [vp, vp, i32p, C.POINTER(C.c_double), C.c_double,
                                                            C.c_double, C.c_double, vp]
    L.cfd_wcns5_euler_step_work_bytes.argtypes = [i32p, C.POINTER(C.c_size_t)]
    L.cfd_c4_viscous_work_bytes.argtypes = [i32p, C.POINTER(C.c_size_t)]
    L.cfd_c4_viscous_add_periodic.argtypes = [vp, vp, vp, C.c_size_t, i32p, C.POINTER(C.c_double), C.c_double,
                                              C.c_double, C.c_double, C.c_double, vp]
    L.cfd_wcns5_euler_steps_periodic.argtypes = [vp, vp, C.c_size_t, i32p, C.POINTER(C.c_double), C.c_double,
                                                 C.c_double, C.c_double, C.c_double, i32, vp]
    L.cfd_wcns5_metrics_periodic.argtypes = [vp, C.POINTER(C.c_double), i32p, vp, vp, vp]
    L.cfd_wcns5_euler_residual_curv_periodic.argtypes = [vp, vp, vp, vp, vp, C.c_size_t, i32p, C.c_double,
                                                         C.c_double, C.c_double, vp]
    L.cfd_wcns5_euler_steps_curv_periodic.argtypes = [vp, vp, vp, vp, C.c_size_t, i32p, C.c_double, C.c_double,
                                                      C.c_double, C.c_double, i32, vp]
    L.cfd_c4_viscous_curv_work_bytes.argtypes = [i32p, C.POINTER(C.c_size_t)]
    L.cfd_c4_viscous_add_curv_periodic.argtypes = [vp, vp, vp, vp, vp, C.c_size_t, i32p, C.c_double, C.c_double,
                                                   C.c_double, C.c_double, vp]
    L.cfd_wcns5_time_step_curv_periodic.argtypes = [vp, vp, vp, i32p, C.c_double, C.c_double, i32, C.c_double,
                                                    C.c_double, C.c_double, vp, vp]
    L.cfd_wcns5_metrics_ext.argtypes = [vp, i32p, vp, vp, vp]
    L.cfd_wcns5_euler_blocks_work_bytes.argtypes = [i32, i32p, i32p, C.POINTER(C.c_size_t)]
    L.cfd_wcns5_euler_residual_blocks.argtypes = [i32, i32p, i32p, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                                  C.POINTER(vp), vp, C.c_size_t, C.c_double, C.c_double, C.c_double,
                                                  vp]
    L.cfd_c4_viscous_blocks_work_bytes.argtypes = [i32, i32p, i32p, C.POINTER(C.c_size_t)]
    L.cfd_c4_viscous_add_blocks.argtypes = [i32, i32p, i32p, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                            C.POINTER(vp), vp, C.c_size_t, C.c_double, C.c_double, C.c_double,
                                            C.c_double, vp]
    L.cfd_wcns5_ns_step_work_bytes.argtypes = [i32p, C.POINTER(C.c_size_t)]
    L.cfd_wcns5_ns_steps_curv_periodic.argtypes = [vp, vp, vp, vp, C.c_size_t, i32p, C.c_double, C.c_double,
                                                   C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, i32,
                                                   vp]
    L.cfd_wcns5_implicit_step_work_bytes.argtypes = [i32p, C.POINTER(C.c_size_t)]
    L.cfd_wcns5_implicit_steps_curv_periodic.argtypes = [vp, vp, vp, vp, C.c_size_t, i32p, C.c_double, C.c_double,
                                                         C.c_double, i32, C.c_double, C.c_double, C.c_double,
                                                         C.c_double, i32, i32, vp]
    L.cfd_wcns5_implicit_blocks_work_bytes.argtypes = [i32, i32p, i32p, C.POINTER(C.c_size_t)]
    L.cfd_wcns5_implicit_steps_blocks.argtypes = [i32, i32p, i32p, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp,
                                                  C.c_size_t, C.c_double, C.c_double, C.c_double, i32, C.c_double,
                                                  C.c_double, C.c_double, C.c_double, i32, i32, vp]
    L.cfd_wcns5_ns_blocks_work_bytes.argtypes = [i32, i32p, i32p, C.POINTER(C.c_size_t)]
    L.cfd_wcns5_ns_steps_blocks.argtypes = [i32, i32p, i32p, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), vp,
                                            C.c_size_t, C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                            C.c_double, C.c_double, i32, vp]
    L.cfd_mg_work_size.argtypes = [C.POINTER(vp), i32, C.POINTER(C.c_size_t)]
    L.cfd_mg_cycles.argtypes = [C.POINTER(vp), C.POINTER(vp), i32, i32, i32, i32, vp, C.c_size_t, vp, vp]
    L.cfd_wcns5_extend_vertices.argtypes = [vp, i32p, i32, C.POINTER(C.c_double), vp, vp]
    L.cfd_wcns5_extend_vertices_mask.argtypes = [vp, i32p, i32, C.POINTER(C.c_double), vp, vp]
    L.cfd_wcns5_fill_ghost_blocks.argtypes = [vp, vp, vp, vp, vp, i32p, i32, i32p, C.c_double,
                                              C.POINTER(C.c_double), vp]
    L.cfd_wcns5_steps_blocks_closed.argtypes = [i32, i32p, i32p, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp),
                                                C.POINTER(WcnsClosure), i32, i32, vp, C.c_size_t, C.c_double,
                                                C.c_double, C.c_double, C.c_double, C.c_double, C.c_double,
                                                C.c_double, i32, vp]
    L.cfd_status_string.argtypes = [i32]
    L.cfd_status_string.restype = C.c_char_p
    L.cfd_last_error.argtypes = [vp]
    L.cfd_last_error.restype = C.c_char_p
    for name in EXPORTS:
        if name not in ("cfd_status_string", "cfd_last_error"):
            getattr(L, name).restype = i32
    _lib = L
    return L


class CfdError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def _check(st, ctx=None):
    if st != CFD_OK:
        msg = lib().cfd_last_error(ctx).decode(errors="replace")
        raise CfdError(st, msg)


def to_params(p) -> ParamsS:
    s = ParamsS()
    for f, _ in ParamsS._fields_:
        setattr(s, f, getattr(p, f))
    return s


def to_dims(dims) -> C.Array:
    arr = (Dims * len(dims))()
    for b, (ni, nj, nk) in enumerate(dims):
        arr[b].ni, arr[b].nj, arr[b].nk = ni, nj, nk
    return arr


def to_conns(conns):
    arr = (ConnS * max(len(conns), 1))()
    for n, c in enumerate(conns):
        a = arr[n]
        a.blk, a.face, a.nbr, a.nbr_face = c.blk, c.face, c.nbr, c.nbr_face
        a.lo[:] = list(c.lo)
        a.hi[:] = list(c.hi)
        a.nbr_lo[:] = list(c.nbr_lo)
        a.shift[:] = [float(v) for v in c.shift]
    return arr


def to_bcs(bcs):
    arr = (BCS * max(len(bcs), 1))()
    for n, b in enumerate(bcs):
        a = arr[n]
        a.blk, a.face, a.kind = b.blk, b.face, b.kind
        a.lo[:] = list(b.lo)
        a.hi[:] = list(b.hi)
        a.mach = float(getattr(b, "mach", 0.0))
    return arr


def layout(dims):
    L = lib()
    nb = len(dims)
    off = (C.c_int64 * nb)()
    strd = (C.c_int64 * (4 * nb))()
    tot = C.c_int64()
    _check(L.cfd_layout(nb, to_dims(dims), NG, off, strd, C.byref(tot)))
    return list(off), [tuple(strd[4 * b:4 * b + 4]) for b in range(nb)], int(tot.value)


def _stream_handle(torch, stream):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _scratch(torch, nbytes, device, stream):
    """Temporary device workspace for one call on `stream`.  The caching
    allocator ties a block to the stream current at allocation; when the call
    runs on another stream the block is recorded there too, so that it is not
    handed out again before that stream's work on it has finished."""
    t = torch.empty(nbytes, dtype=torch.uint8, device=device)
    if stream is not None and stream != torch.cuda.current_stream(device):
        t.record_stream(stream)
    return t


def staggered_diff6(f, n, d: int, h: float, out=None, stream=None):
    """Eq. (2) of Section 2.2 on the device (cfd_staggered_diff6): f is a
    contiguous FP64 CUDA tensor [nvar, Nk, Nj, Ni] of face values with
    n[d] + 5 entries along direction d; returns [nvar, nk, nj, ni]."""
    import torch
    ni, nj, nk = (int(v) for v in n)
    if f.dtype != torch.float64 or not f.is_cuda or not f.is_contiguous():
        raise ValueError("f must be a contiguous float64 CUDA tensor")
    want = [f.shape[0], nk + 5 * (d == 2), nj + 5 * (d == 1), ni + 5 * (d == 0)]
    if list(f.shape) != want:
        raise ValueError(f"f has shape {tuple(f.shape)}, expected {tuple(want)}")
    if out is None:
        out = torch.empty((f.shape[0], nk, nj, ni), dtype=torch.float64, device=f.device)
    elif list(out.shape) != [f.shape[0], nk, nj, ni] or out.dtype != torch.float64 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float64 tensor [nvar, nk, nj, ni]")
    nn = (C.c_int32 * 3)(ni, nj, nk)
    _check(lib().cfd_staggered_diff6(_ptr(f), _ptr(out), nn, int(d), int(f.shape[0]), float(h),
                                     _stream_handle(torch, stream)))
    return out


def wcns5_edges(u, n, d: int, eps: float = 1e-6, stream=None):
    """WCNS-E-5 face states on the device (cfd_wcns5_edges): u is a contiguous
    FP64 CUDA tensor [nvar, Nk, Nj, Ni] of cell values with n[d] + 10 entries
    along direction d; returns (left, right), each with n[d] + 5 faces along d."""
    import torch
    ni, nj, nk = (int(v) for v in n)
    if u.dtype != torch.float64 or not u.is_cuda or not u.is_contiguous():
        raise ValueError("u must be a contiguous float64 CUDA tensor")
    want = [u.shape[0], nk + 10 * (d == 2), nj + 10 * (d == 1), ni + 10 * (d == 0)]
    if list(u.shape) != want:
        raise ValueError(f"u has shape {tuple(u.shape)}, expected {tuple(want)}")
    fshape = [u.shape[0], nk + 5 * (d == 2), nj + 5 * (d == 1), ni + 5 * (d == 0)]
    left = torch.empty(fshape, dtype=torch.float64, device=u.device)
    right = torch.empty(fshape, dtype=torch.float64, device=u.device)
    nn = (C.c_int32 * 3)(ni, nj, nk)
    _check(lib().cfd_wcns5_edges(_ptr(u), _ptr(left), _ptr(right), nn, int(d), int(u.shape[0]), float(eps),
                                 _stream_handle(torch, stream)))
    return left, right


def wcns5_euler_residual_periodic(q, h, gamma: float = 1.4, entropy_fix: float = 0.1, eps: float = 1e-6,
                                  out=None, work=None, stream=None):
    """Inviscid WCNS-E-5 residual of a periodic Cartesian block on the device
    (cfd_wcns5_euler_residual_periodic): q is a contiguous FP64 CUDA tensor
    [5, nk, nj, ni]; returns R of the same shape (dQ/dt = -R)."""
    import torch
    if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
        raise ValueError("q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
    nk, nj, ni = (int(v) for v in q.shape[1:])
    nn = (C.c_int32 * 3)(ni, nj, nk)
    nbytes = C.c_size_t()
    _check(lib().cfd_wcns5_euler_work_bytes(nn, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, q.device, stream)
    if out is None:
        out = torch.empty_like(q)
    hh = (C.c_double * 3)(*[float(v) for v in h])
    _check(lib().cfd_wcns5_euler_residual_periodic(_ptr(q), _ptr(out), _ptr(work), nbytes.value, nn, hh,
                                                   float(gamma), float(entropy_fix), float(eps),
                                                   _stream_handle(torch, stream)))
    return out


def wcns5_euler_residual_periodic_noalloc(q, h, out, gamma: float = 1.4, entropy_fix: float = 0.1,
                                          eps: float = 1e-6, stream=None):
    """The residual of wcns5_euler_residual_periodic through the entry point
    that allocates nothing (cfd_wcns5_euler_residual_periodic_noalloc): its
    scratch is the library's static device array, so no workspace is passed
    and `out` (contiguous FP64 CUDA tensor shaped like q) must be given."""
    import torch
    if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
        raise ValueError("q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
    if out.shape != q.shape or out.dtype != torch.float64 or not out.is_contiguous() or out.device != q.device:
        raise ValueError("out must be a contiguous float64 tensor shaped like q on its device")
    nk, nj, ni = (int(v) for v in q.shape[1:])
    nn = (C.c_int32 * 3)(ni, nj, nk)
    hh = (C.c_double * 3)(*[float(v) for v in h])
    _check(lib().cfd_wcns5_euler_residual_periodic_noalloc(_ptr(q), _ptr(out), nn, hh, float(gamma),
                                                           float(entropy_fix), float(eps),
                                                           _stream_handle(torch, stream)))
    return out


def wcns5_euler_steps_periodic(q, h, dt: float, nsteps: int, gamma: float = 1.4, entropy_fix: float = 0.1,
                               eps: float = 1e-6, work=None, stream=None):
    """nsteps RK3 steps of the periodic WCNS-E-5 Euler residual on the device,
    in place on q (contiguous FP64 CUDA tensor [5, nk, nj, ni]); returns q."""
    import torch
    if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
        raise ValueError("q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
    nk, nj, ni = (int(v) for v in q.shape[1:])
    nn = (C.c_int32 * 3)(ni, nj, nk)
    nbytes = C.c_size_t()
    _check(lib().cfd_wcns5_euler_step_work_bytes(nn, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, q.device, stream)
    hh = (C.c_double * 3)(*[float(v) for v in h])
    _check(lib().cfd_wcns5_euler_steps_periodic(_ptr(q), _ptr(work), nbytes.value, nn, hh, float(gamma),
                                                float(entropy_fix), float(eps), float(dt), int(nsteps),
                                                _stream_handle(torch, stream)))
    return q


def c4_viscous_add_periodic(q, r, h, gamma: float = 1.4, prandtl: float = 0.72, mu_inf: float = 1e-3,
                            s_star: float = 110.4 / 288.15, work=None, stream=None):
    """Adds -div F_v (fourth-order central, periodic Cartesian block) to r on
    the device (cfd_c4_viscous_add_periodic); q, r: contiguous FP64 CUDA
    tensors [5, nk, nj, ni].  Returns r."""
    import torch
    for t in (q, r):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 4 or t.shape[0] != 5:
            raise ValueError("q and r must be contiguous float64 CUDA tensors [5, nk, nj, ni]")
    nk, nj, ni = (int(v) for v in q.shape[1:])
    nn = (C.c_int32 * 3)(ni, nj, nk)
    nbytes = C.c_size_t()
    _check(lib().cfd_c4_viscous_work_bytes(nn, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, q.device, stream)
    hh = (C.c_double * 3)(*[float(v) for v in h])
    _check(lib().cfd_c4_viscous_add_periodic(_ptr(q), _ptr(r), _ptr(work), nbytes.value, nn, hh, float(gamma),
                                             float(prandtl), float(mu_inf), float(s_star),
                                             _stream_handle(torch, stream)))
    return r


def wcns5_metrics_periodic(xv, period, stream=None):
    """Metrics of a periodic curvilinear block on the device
    (cfd_wcns5_metrics_periodic): xv is a contiguous FP64 CUDA tensor
    [3, nk, nj, ni] of vertex coordinates (vertex (i, j, k) = the upper corner
    of cell (i, j, k)); period[d] the grid's displacement over one period
    along direction d (3 x 3).  Returns (S [3, 3, nk, nj, ni], Jinv [nk, nj, ni])."""
    import torch
    if xv.dtype != torch.float64 or not xv.is_cuda or not xv.is_contiguous() or xv.dim() != 4 or xv.shape[0] != 3:
        raise ValueError("xv must be a contiguous float64 CUDA tensor [3, nk, nj, ni]")
    nk, nj, ni = (int(v) for v in xv.shape[1:])
    per = [float(v) for row in period for v in row]
    if len(per) != 9:
        raise ValueError("period must be 3 x 3")
    S = torch.empty((3, 3, nk, nj, ni), dtype=torch.float64, device=xv.device)
    jinv = torch.empty((nk, nj, ni), dtype=torch.float64, device=xv.device)
    _check(lib().cfd_wcns5_metrics_periodic(_ptr(xv), (C.c_double * 9)(*per), (C.c_int32 * 3)(ni, nj, nk), _ptr(S),
                                            _ptr(jinv), _stream_handle(torch, stream)))
    return S, jinv


def wcns5_euler_residual_curv_periodic(q, S, jinv, gamma: float = 1.4, entropy_fix: float = 0.1, eps: float = 1e-6,
                                       out=None, work=None, stream=None):
    """Inviscid WCNS-E-5 residual of a periodic curvilinear block on the device
    (cfd_wcns5_euler_residual_curv_periodic): q [5, nk, nj, ni], S and jinv
    from wcns5_metrics_periodic, all contiguous FP64 CUDA tensors; returns R
    (dQ/dt = -R)."""
    import torch
    if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
        raise ValueError("q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
    nk, nj, ni = (int(v) for v in q.shape[1:])
    for t, shp in ((S, (3, 3, nk, nj, ni)), (jinv, (nk, nj, ni))):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
            raise ValueError("S and jinv must be contiguous float64 CUDA tensors of the block's shape")
    nn = (C.c_int32 * 3)(ni, nj, nk)
    nbytes = C.c_size_t()
    _check(lib().cfd_wcns5_euler_work_bytes(nn, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, q.device, stream)
    if out is None:
        out = torch.empty_like(q)
    _check(lib().cfd_wcns5_euler_residual_curv_periodic(_ptr(q), _ptr(S), _ptr(jinv), _ptr(out), _ptr(work),
                                                        nbytes.value, nn, float(gamma), float(entropy_fix),
                                                        float(eps), _stream_handle(torch, stream)))
    return out


def wcns5_euler_steps_curv_periodic(q, S, jinv, dt: float, nsteps: int, gamma: float = 1.4,
                                    entropy_fix: float = 0.1, eps: float = 1e-6, work=None, stream=None):
    """nsteps RK3 steps of the curvilinear periodic WCNS-E-5 Euler residual on
    the device, in place on q (contiguous FP64 CUDA tensor [5, nk, nj, ni]);
    S, jinv from wcns5_metrics_periodic.  Returns q."""
    import torch
    if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
        raise ValueError("q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
    nk, nj, ni = (int(v) for v in q.shape[1:])
    for t, shp in ((S, (3, 3, nk, nj, ni)), (jinv, (nk, nj, ni))):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
            raise ValueError("S and jinv must be contiguous float64 CUDA tensors of the block's shape")
    nn = (C.c_int32 * 3)(ni, nj, nk)
    nbytes = C.c_size_t()
    _check(lib().cfd_wcns5_euler_step_work_bytes(nn, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, q.device, stream)
    _check(lib().cfd_wcns5_euler_steps_curv_periodic(_ptr(q), _ptr(S), _ptr(jinv), _ptr(work), nbytes.value, nn,
                                                     float(gamma), float(entropy_fix), float(eps), float(dt),
                                                     int(nsteps), _stream_handle(torch, stream)))
    return q


def c4_viscous_add_curv_periodic(q, r, S, jinv, gamma: float = 1.4, prandtl: float = 0.72, mu_inf: float = 1e-3,
                                 s_star: float = 110.4 / 288.15, work=None, stream=None):
    """Adds -div F_v (fourth-order central, periodic curvilinear block) to r on
    the device (cfd_c4_viscous_add_curv_periodic); q, r [5, nk, nj, ni], S and
    jinv from wcns5_metrics_periodic, all contiguous FP64 CUDA tensors.
    Returns r."""
    import torch
    for t in (q, r):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 4 or t.shape[0] != 5:
            raise ValueError("q and r must be contiguous float64 CUDA tensors [5, nk, nj, ni]")
    nk, nj, ni = (int(v) for v in q.shape[1:])
    for t, shp in ((S, (3, 3, nk, nj, ni)), (jinv, (nk, nj, ni))):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
            raise ValueError("S and jinv must be contiguous float64 CUDA tensors of the block's shape")
    nn = (C.c_int32 * 3)(ni, nj, nk)
    nbytes = C.c_size_t()
    _check(lib().cfd_c4_viscous_curv_work_bytes(nn, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, q.device, stream)
    _check(lib().cfd_c4_viscous_add_curv_periodic(_ptr(q), _ptr(S), _ptr(jinv), _ptr(r), _ptr(work), nbytes.value,
                                                  nn, float(gamma), float(prandtl), float(mu_inf), float(s_star),
                                                  _stream_handle(torch, stream)))
    return r


def wcns5_time_step_curv_periodic(q, S, jinv, cfl: float, gamma: float = 1.4, viscous: bool = False,
                                   prandtl: float = 0.72, mu_inf: float = 1e-3, s_star: float = 110.4 / 288.15,
                                   out=None, stream=None):
    """The global CFL time step of a periodic curvilinear block on the device
    (cfd_wcns5_time_step_curv_periodic).  Returns a one-element FP64 CUDA
    tensor (out, if given), filled asynchronously on the stream."""
    import torch
    if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
        raise ValueError("q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
    nk, nj, ni = (int(v) for v in q.shape[1:])
    for t, shp in ((S, (3, 3, nk, nj, ni)), (jinv, (nk, nj, ni))):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
            raise ValueError("S and jinv must be contiguous float64 CUDA tensors of the block's shape")
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=q.device)
    _check(lib().cfd_wcns5_time_step_curv_periodic(_ptr(q), _ptr(S), _ptr(jinv), (C.c_int32 * 3)(ni, nj, nk),
                                                   float(gamma), float(cfl), 1 if viscous else 0, float(prandtl),
                                                   float(mu_inf), float(s_star), _ptr(out),
                                                   _stream_handle(torch, stream)))
    return out


def wcns5_metrics_ext(xe, stream=None):
    """Metrics of a block from its vertices -3 .. n + 1 along each direction
    (cfd_wcns5_metrics_ext): xe a contiguous FP64 CUDA tensor
    [3, nk + 5, nj + 5, ni + 5].  Returns (S [3, 3, nk, nj, ni], Jinv)."""
    import torch
    if xe.dtype != torch.float64 or not xe.is_cuda or not xe.is_contiguous() or xe.dim() != 4 or xe.shape[0] != 3:
        raise ValueError("xe must be a contiguous float64 CUDA tensor [3, nk + 5, nj + 5, ni + 5]")
    nk, nj, ni = (int(v) - 5 for v in xe.shape[1:])
    if min(nk, nj, ni) < 1:
        raise ValueError("xe must hold at least one cell along each direction")
    S = torch.empty((3, 3, nk, nj, ni), dtype=torch.float64, device=xe.device)
    jinv = torch.empty((nk, nj, ni), dtype=torch.float64, device=xe.device)
    _check(lib().cfd_wcns5_metrics_ext(_ptr(xe), (C.c_int32 * 3)(ni, nj, nk), _ptr(S), _ptr(jinv),
                                       _stream_handle(torch, stream)))
    return S, jinv


def wcns5_euler_residual_blocks(qs, Ss, jinvs, nbr, gamma: float = 1.4, entropy_fix: float = 0.1, eps: float = 1e-6,
                                outs=None, work=None, stream=None):
    """The curvilinear WCNS-E-5 residual of blocks joined face to face
    (cfd_wcns5_euler_residual_blocks): per block q [5, nk, nj, ni], S, jinv
    (contiguous FP64 CUDA tensors); nbr[b][2d + side] the block across face
    (d, side).  Returns the residuals."""
    import torch
    nblk = len(qs)
    dims = (C.c_int32 * (3 * nblk))()
    for b, q in enumerate(qs):
        if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
            raise ValueError("every q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
        nk, nj, ni = (int(v) for v in q.shape[1:])
        dims[3 * b:3 * b + 3] = [ni, nj, nk]
        for t, shp in ((Ss[b], (3, 3, nk, nj, ni)), (jinvs[b], (nk, nj, ni))):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
                raise ValueError("S and jinv must be contiguous float64 CUDA tensors of each block's shape")
    nb = (C.c_int32 * (6 * nblk))(*[int(v) for row in nbr for v in row])
    nbytes = C.c_size_t()
    _check(lib().cfd_wcns5_euler_blocks_work_bytes(nblk, dims, nb, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, max(nbytes.value, 8), qs[0].device, stream)
    if outs is None:
        outs = [torch.empty_like(q) for q in qs]
    ptrs = lambda ts: (C.c_void_p * nblk)(*[_ptr(t) for t in ts])   # noqa: E731
    _check(lib().cfd_wcns5_euler_residual_blocks(nblk, dims, nb, ptrs(qs), ptrs(Ss), ptrs(jinvs), ptrs(outs),
                                                 _ptr(work), nbytes.value, float(gamma), float(entropy_fix),
                                                 float(eps), _stream_handle(torch, stream)))
    return outs


def c4_viscous_add_blocks(qs, rs, Ss, jinvs, nbr, gamma: float = 1.4, prandtl: float = 0.72, mu_inf: float = 1e-3,
                          s_star: float = 110.4 / 288.15, work=None, stream=None):
    """Adds the fourth-order viscous terms of blocks joined face to face to
    their residuals on the device (cfd_c4_viscous_add_blocks); per block q, r
    [5, nk, nj, ni], S, jinv (contiguous FP64 CUDA tensors); nbr as for
    wcns5_euler_residual_blocks.  Returns rs."""
    import torch
    nblk = len(qs)
    dims = (C.c_int32 * (3 * nblk))()
    for b, (q, r) in enumerate(zip(qs, rs)):
        for t in (q, r):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.dim() != 4 or t.shape[0] != 5:
                raise ValueError("every q and r must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
        nk, nj, ni = (int(v) for v in q.shape[1:])
        if tuple(r.shape[1:]) != (nk, nj, ni):
            raise ValueError("r must have its block's shape")
        dims[3 * b:3 * b + 3] = [ni, nj, nk]
        for t, shp in ((Ss[b], (3, 3, nk, nj, ni)), (jinvs[b], (nk, nj, ni))):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
                raise ValueError("S and jinv must be contiguous float64 CUDA tensors of each block's shape")
    nb = (C.c_int32 * (6 * nblk))(*[int(v) for row in nbr for v in row])
    nbytes = C.c_size_t()
    _check(lib().cfd_c4_viscous_blocks_work_bytes(nblk, dims, nb, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, qs[0].device, stream)
    ptrs = lambda ts: (C.c_void_p * nblk)(*[_ptr(t) for t in ts])   # noqa: E731
    _check(lib().cfd_c4_viscous_add_blocks(nblk, dims, nb, ptrs(qs), ptrs(Ss), ptrs(jinvs), ptrs(rs), _ptr(work),
                                           nbytes.value, float(gamma), float(prandtl), float(mu_inf), float(s_star),
                                           _stream_handle(torch, stream)))
    return rs


def wcns5_ns_steps_curv_periodic(q, S, jinv, dt: float, nsteps: int, gamma: float = 1.4, entropy_fix: float = 0.1,
                                 eps: float = 1e-6, prandtl: float = 0.72, mu_inf: float = 1e-3,
                                 s_star: float = 110.4 / 288.15, work=None, stream=None):
    """nsteps RK3 Navier-Stokes steps on a periodic curvilinear block on the
    device (cfd_wcns5_ns_steps_curv_periodic), in place on q (contiguous FP64
    CUDA tensor [5, nk, nj, ni]); S, jinv from wcns5_metrics_periodic.
    Returns q."""
    import torch
    if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
        raise ValueError("q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
    nk, nj, ni = (int(v) for v in q.shape[1:])
    for t, shp in ((S, (3, 3, nk, nj, ni)), (jinv, (nk, nj, ni))):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
            raise ValueError("S and jinv must be contiguous float64 CUDA tensors of the block's shape")
    nn = (C.c_int32 * 3)(ni, nj, nk)
    nbytes = C.c_size_t()
    _check(lib().cfd_wcns5_ns_step_work_bytes(nn, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, q.device, stream)
    _check(lib().cfd_wcns5_ns_steps_curv_periodic(_ptr(q), _ptr(S), _ptr(jinv), _ptr(work), nbytes.value, nn,
                                                  float(gamma), float(entropy_fix), float(eps), float(prandtl),
                                                  float(mu_inf), float(s_star), float(dt), int(nsteps),
                                                  _stream_handle(torch, stream)))
    return q


def wcns5_implicit_steps_curv_periodic(q, S, jinv, dt: float, nsteps: int, sweeps: int, gamma: float = 1.4,
                                       entropy_fix: float = 0.1, eps: float = 1e-6, viscous: bool = False,
                                       prandtl: float = 0.72, mu_inf: float = 1e-3, s_star: float = 110.4 / 288.15,
                                       work=None, stream=None):
    """nsteps implicit steps (backward Euler, point-Jacobi sweeps) of the
    curvilinear periodic WCNS-E-5 residual, with the fourth-order viscous
    terms when viscous, on the device (cfd_wcns5_implicit_steps_curv_periodic),
    in place on q.  Returns q."""
    import torch
    if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
        raise ValueError("q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
    nk, nj, ni = (int(v) for v in q.shape[1:])
    for t, shp in ((S, (3, 3, nk, nj, ni)), (jinv, (nk, nj, ni))):
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
            raise ValueError("S and jinv must be contiguous float64 CUDA tensors of the block's shape")
    nn = (C.c_int32 * 3)(ni, nj, nk)
    nbytes = C.c_size_t()
    _check(lib().cfd_wcns5_implicit_step_work_bytes(nn, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, q.device, stream)
    _check(lib().cfd_wcns5_implicit_steps_curv_periodic(_ptr(q), _ptr(S), _ptr(jinv), _ptr(work), nbytes.value, nn,
                                                        float(gamma), float(entropy_fix), float(eps),
                                                        1 if viscous else 0, float(prandtl), float(mu_inf),
                                                        float(s_star), float(dt), int(nsteps), int(sweeps),
                                                        _stream_handle(torch, stream)))
    return q


def wcns5_implicit_steps_blocks(qs, Ss, jinvs, nbr, dt: float, nsteps: int, sweeps: int, gamma: float = 1.4,
                                entropy_fix: float = 0.1, eps: float = 1e-6, viscous: bool = False,
                                prandtl: float = 0.72, mu_inf: float = 1e-3, s_star: float = 110.4 / 288.15,
                                work=None, stream=None):
    """Implicit steps (viscous optional) on blocks joined face to face on the device
    (cfd_wcns5_implicit_steps_blocks), in place on every q; per block q, S,
    jinv contiguous FP64 CUDA tensors; nbr as for
    wcns5_euler_residual_blocks.  Returns qs."""
    import torch
    nblk = len(qs)
    dims = (C.c_int32 * (3 * nblk))()
    for b, q in enumerate(qs):
        if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
            raise ValueError("every q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
        nk, nj, ni = (int(v) for v in q.shape[1:])
        dims[3 * b:3 * b + 3] = [ni, nj, nk]
        for t, shp in ((Ss[b], (3, 3, nk, nj, ni)), (jinvs[b], (nk, nj, ni))):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
                raise ValueError("S and jinv must be contiguous float64 CUDA tensors of each block's shape")
    nb = (C.c_int32 * (6 * nblk))(*[int(v) for row in nbr for v in row])
    nbytes = C.c_size_t()
    _check(lib().cfd_wcns5_implicit_blocks_work_bytes(nblk, dims, nb, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, qs[0].device, stream)
    ptrs = lambda ts: (C.c_void_p * nblk)(*[_ptr(t) for t in ts])   # noqa: E731
    _check(lib().cfd_wcns5_implicit_steps_blocks(nblk, dims, nb, ptrs(qs), ptrs(Ss), ptrs(jinvs), _ptr(work),
                                                 nbytes.value, float(gamma), float(entropy_fix), float(eps),
                                                 1 if viscous else 0, float(prandtl), float(mu_inf), float(s_star),
                                                 float(dt), int(nsteps), int(sweeps), _stream_handle(torch, stream)))
    return qs


def wcns5_ns_steps_blocks(qs, Ss, jinvs, nbr, dt: float, nsteps: int, gamma: float = 1.4, entropy_fix: float = 0.1,
                          eps: float = 1e-6, prandtl: float = 0.72, mu_inf: float = 1e-3,
                          s_star: float = 110.4 / 288.15, work=None, stream=None):
    """RK3 Navier-Stokes steps on blocks joined face to face on the device
    (cfd_wcns5_ns_steps_blocks), in place on every q; per block q, S, jinv
    contiguous FP64 CUDA tensors; nbr as for wcns5_euler_residual_blocks.
    Returns qs."""
    import torch
    nblk = len(qs)
    dims = (C.c_int32 * (3 * nblk))()
    for b, q in enumerate(qs):
        if q.dtype != torch.float64 or not q.is_cuda or not q.is_contiguous() or q.dim() != 4 or q.shape[0] != 5:
            raise ValueError("every q must be a contiguous float64 CUDA tensor [5, nk, nj, ni]")
        nk, nj, ni = (int(v) for v in q.shape[1:])
        dims[3 * b:3 * b + 3] = [ni, nj, nk]
        for t, shp in ((Ss[b], (3, 3, nk, nj, ni)), (jinvs[b], (nk, nj, ni))):
            if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != shp:
                raise ValueError("S and jinv must be contiguous float64 CUDA tensors of each block's shape")
    nb = (C.c_int32 * (6 * nblk))(*[int(v) for row in nbr for v in row])
    nbytes = C.c_size_t()
    _check(lib().cfd_wcns5_ns_blocks_work_bytes(nblk, dims, nb, C.byref(nbytes)))
    if work is None or work.numel() * work.element_size() < nbytes.value:
        work = _scratch(torch, nbytes.value, qs[0].device, stream)
    ptrs = lambda ts: (C.c_void_p * nblk)(*[_ptr(t) for t in ts])   # noqa: E731
    _check(lib().cfd_wcns5_ns_steps_blocks(nblk, dims, nb, ptrs(qs), ptrs(Ss), ptrs(jinvs), _ptr(work), nbytes.value,
                                           float(gamma), float(entropy_fix), float(eps), float(prandtl),
                                           float(mu_inf), float(s_star), float(dt), int(nsteps),
                                           _stream_handle(torch, stream)))
    return qs



class Multigrid:
    """Multigrid V-cycles (cfd_mg_cycles) for a solver's steady march: the
    solver's grid and nlevels - 1 coarsenings (cases.hierarchy), each level a
    Solver of its own whose state is a working state of the cycle."""

    def __init__(self, solver, nlevels: int = 3, pre: int = 1, coarse: int = 2):
        from . import cases as _cases
        torch = solver.torch
        self.torch = torch
        self.solver = solver
        self.pre, self.coarse = int(pre), int(coarse)
        hier = _cases.hierarchy(solver.case, nlevels)
        self.levels = [solver] + [Solver(c, device=str(solver.device), stream=solver.stream) for c in hier[1:]]
        self._ctx = (C.c_void_p * nlevels)(*[lv.ctx.value for lv in self.levels])
        nb = C.c_size_t()
        _check(lib().cfd_mg_work_size(self._ctx, nlevels, C.byref(nb)))
        self._work = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=solver.device)
        base = self._work.data_ptr()
        self._w = C.c_void_p(base + (-base) % 256)
        self._wb = C.c_size_t(int(nb.value))

    def cycles(self, n: int, hist: bool = True, arena=None):
        """n V-cycles in place on the solver's state (or arena); returns the
        history [n, 12] (device) or None."""
        torch = self.torch
        q0 = self.solver.q if arena is None else arena
        qs = (C.c_void_p * len(self.levels))(*([_ptr(q0)] + [_ptr(lv.q) for lv in self.levels[1:]]))
        h = torch.zeros((n, 12), dtype=torch.float64, device=self.solver.device) if hist and n > 0 else None
        _check(lib().cfd_mg_cycles(self._ctx, qs, len(self.levels), self.pre, self.coarse, int(n), self._w, self._wb,
                                   _ptr(h) if h is not None else None, self.solver._s()), self.solver.ctx)
        return h

    def close(self):
        for lv in self.levels[1:]:
            lv.close()
        self.levels = self.levels[:1]


WCNS5_GHOST = 5
WCNS5_XLAYERS = 7


def wcns5_extend_vertices(xv, bounded: int, period, stream=None):
    """Vertices for the closures (cfd_wcns5_extend_vertices): xv a contiguous
    FP64 CUDA tensor [3, nk', nj', ni'] (n_d upper corners along periodic
    directions, n_d + 1 planes along `bounded`), period [3][3] the
    displacement over one period per direction.  Returns the extended
    vertices [3, Ek, Ej, Ei]."""
    import torch
    if xv.dtype != torch.float64 or not xv.is_cuda or not xv.is_contiguous() or xv.dim() != 4 or xv.shape[0] != 3:
        raise ValueError("xv must be a contiguous float64 CUDA tensor [3, nk', nj', ni']")
    n = [int(xv.shape[3]), int(xv.shape[2]), int(xv.shape[1])]
    if bounded in (0, 1, 2):
        n[bounded] -= 1
    e = [n[d] + 1 + 2 * WCNS5_XLAYERS if d == bounded else n[d] + 5 for d in range(3)]
    xe = torch.empty((3, e[2], e[1], e[0]), dtype=torch.float64, device=xv.device)
    per = (C.c_double * 9)(*[float(v) for row in period for v in row])
    _check(lib().cfd_wcns5_extend_vertices(_ptr(xv), (C.c_int32 * 3)(*n), int(bounded), per, _ptr(xe),
                                           _stream_handle(torch, stream)))
    return xe


def wcns5_fill_ghost_blocks(q, q_lo, q_hi, S, S_lo, bounded: int, kinds, uinf, gamma: float = 1.4, stream=None):
    """Ghost-block states from the owner's state (cfd_wcns5_fill_ghost_blocks),
    in place on q_lo and q_hi."""
    import torch
    nk, nj, ni = (int(v) for v in q.shape[1:])
    _check(lib().cfd_wcns5_fill_ghost_blocks(_ptr(q), _ptr(q_lo), _ptr(q_hi), _ptr(S), _ptr(S_lo),
                                             (C.c_int32 * 3)(ni, nj, nk), int(bounded),
                                             (C.c_int32 * 2)(*[int(k) for k in kinds]), float(gamma),
                                             (C.c_double * 3)(*[float(u) for u in uinf]),
                                             _stream_handle(torch, stream)))


class WcnsClosedTiling:
    """Owner blocks tiling the two periodic directions of a curvilinear grid
    whose two faces across the third (`bounded`) are walls or the far field,
    each owner closed by its two ghost blocks (cfd_wcns5_extend_vertices,
    cfd_wcns5_metrics_ext, cfd_wcns5_fill_ghost_blocks, the joined-block
    residual, viscous terms and RK3 steps).  xv: the whole grid's vertices as
    for wcns5_extend_vertices (a CUDA tensor); cuts[d] for the periodic d: the
    block boundaries 0 = c_0 < ... < c_m = n_d (default: one owner); kinds: the
    cfd_bc_kind of the low and high face; uinf: the far-field velocity.
    Owners are numbered along the first periodic direction fastest; block
    3 o + r of the tables is owner o (r = 0) or its low (1) or high (2) ghost
    block."""

    def __init__(self, xv, period, bounded: int, kinds, uinf=(0.0, 0.0, 0.0), gamma: float = 1.4, cuts=None,
                 stream=None):
        import torch
        self.torch = torch
        self.stream = stream
        self.bounded, self.kinds, self.uinf, self.gamma = int(bounded), tuple(kinds), tuple(uinf), float(gamma)
        d = self.bounded
        N = [int(xv.shape[3]), int(xv.shape[2]), int(xv.shape[1])]
        N[d] -= 1
        self.N = tuple(N)
        per = [t for t in range(3) if t != d]
        cuts = dict(cuts or {})
        cuts = {t: [int(v) for v in cuts.get(t, [0, N[t]])] for t in per}
        for t in per:
            c = cuts[t]
            if c[0] != 0 or c[-1] != N[t] or any(b <= a for a, b in zip(c, c[1:])):
                raise ValueError(f"bad cuts along direction {t}: {c}")
        m0, m1 = len(cuts[per[0]]) - 1, len(cuts[per[1]]) - 1
        self.owners = []
        for b1 in range(m1):
            for b0 in range(m0):
                lo, ext = [0, 0, 0], list(N)
                for t, b in ((per[0], b0), (per[1], b1)):
                    lo[t], ext[t] = cuts[t][b], cuts[t][b + 1] - cuts[t][b]
                self.owners.append((tuple(lo), tuple(ext)))
        no = len(self.owners)
        self.dims, nbr = [], [[0] * 6 for _ in range(3 * no)]
        for o, (lo, ext) in enumerate(self.owners):
            g = list(ext)
            g[d] = WCNS5_GHOST
            self.dims += [tuple(ext), tuple(g), tuple(g)]
            b0, b1 = o % m0, o // m0
            for t, (pos, m) in zip(per, ((b0, m0), (b1, m1))):
                for side in (0, 1):
                    pn = (pos + (-1 if side == 0 else 1)) % m
                    on = pn + b1 * m0 if t == per[0] else b0 + pn * m0
                    for r in range(3):
                        nbr[3 * o + r][2 * t + side] = 3 * on + r
            B = 2 * d
            nbr[3 * o][B], nbr[3 * o + 1][B + 1] = 3 * o + 1, 3 * o
            nbr[3 * o][B + 1], nbr[3 * o + 2][B] = 3 * o + 2, 3 * o
            nbr[3 * o + 1][B], nbr[3 * o + 2][B + 1] = 3 * o + 2, 3 * o + 1
        self.nbr = nbr
        xe = wcns5_extend_vertices(xv, d, period, stream)
        org = [3, 3, 3]
        org[d] = WCNS5_XLAYERS + 1
        self.S, self.jinv = [], []
        for lo, ext in self.owners:
            for start, cnt in ((0, N[d]), (-WCNS5_GHOST, WCNS5_GHOST), (N[d], WCNS5_GHOST)):
                sl = []
                for a in (2, 1, 0):
                    if a == d:
                        sl.append(slice(org[a] - 3 + start, org[a] - 3 + start + cnt + 5))
                    else:
                        sl.append(slice(org[a] - 3 + lo[a], org[a] - 3 + lo[a] + ext[a] + 5))
                S, J = wcns5_metrics_ext(xe[(slice(None),) + tuple(sl)].contiguous(), stream)
                self.S.append(S)
                self.jinv.append(J)
        self.ghosts = [torch.zeros((5, g[2], g[1], g[0]), dtype=torch.float64, device=xv.device)
                       for o in range(no) for g in self.dims[3 * o + 1:3 * o + 3]]

    def split(self, q):
        """The owners' states (contiguous copies) cut from a whole-grid state."""
        out = []
        for lo, ext in self.owners:
            sl = [slice(None)] + [slice(lo[a], lo[a] + ext[a]) for a in (2, 1, 0)]
            out.append(q[tuple(sl)].contiguous())
        return out

    def _all(self, qs):
        return [x for o, q in enumerate(qs) for x in (q, self.ghosts[2 * o], self.ghosts[2 * o + 1])]

    def _fill_all(self, qs):
        for o, q in enumerate(qs):
            wcns5_fill_ghost_blocks(q, self.ghosts[2 * o], self.ghosts[2 * o + 1], self.S[3 * o], self.S[3 * o + 1],
                                    self.bounded, self.kinds, self.uinf, self.gamma, self.stream)

    def fill(self, qs):
        """The ghost blocks' states from the owners' states."""
        self._fill_all(qs)

    def residual(self, qs, entropy_fix: float = 0.1, eps: float = 1e-6, viscous=None):
        """R of every owner (dQ/dt = -R); viscous = (prandtl, mu_inf, s_star) adds
        the fourth-order viscous terms."""
        self._fill_all(qs)
        allq = self._all(qs)
        rs = wcns5_euler_residual_blocks(allq, self.S, self.jinv, self.nbr, self.gamma, entropy_fix, eps,
                                         stream=self.stream)
        if viscous is not None:
            c4_viscous_add_blocks(allq, rs, self.S, self.jinv, self.nbr, self.gamma, *viscous, stream=self.stream)
        return [rs[3 * o] for o in range(len(qs))]

    def steps(self, qs, dt: float, nsteps: int, entropy_fix: float = 0.1, eps: float = 1e-6, viscous=None,
              work=None):
        """nsteps RK3 steps in place on the owners' states (cfd_wcns5_steps_blocks_closed)."""
        torch = self.torch
        allq = self._all(qs)
        nb = len(allq)
        dims = (C.c_int32 * (3 * nb))(*[v for m in self.dims for v in m])
        nbt = (C.c_int32 * (6 * nb))(*[v for row in self.nbr for v in row])
        nbytes = C.c_size_t()
        _check(lib().cfd_wcns5_ns_blocks_work_bytes(nb, dims, nbt, C.byref(nbytes)))
        if work is None or work.numel() * work.element_size() < nbytes.value:
            work = _scratch(torch, nbytes.value, qs[0].device, self.stream)
        no = len(qs)
        cls = (WcnsClosure * no)(*[WcnsClosure(3 * o, 3 * o + 1, 3 * o + 2, self.bounded,
                                               (C.c_int32 * 2)(*self.kinds), (C.c_double * 3)(*self.uinf))
                                   for o in range(no)])
        pr, mu, ss = viscous if viscous is not None else (0.72, 0.0, 110.4 / 288.15)
        ptrs = lambda ts: (C.c_void_p * nb)(*[_ptr(t) for t in ts])   # noqa: E731
        _check(lib().cfd_wcns5_steps_blocks_closed(nb, dims, nbt, ptrs(allq), ptrs(self.S), ptrs(self.jinv), cls, no,
                                                   1 if viscous is not None else 0, _ptr(work), nbytes.value,
                                                   self.gamma, float(entropy_fix), float(eps), float(pr), float(mu),
                                                   float(ss), float(dt), int(nsteps),
                                                   _stream_handle(torch, self.stream)))
        return qs


class WcnsClosedBlock(WcnsClosedTiling):
    """One owner block (the untiled WcnsClosedTiling): the same calls on a
    single state q instead of a list; S, jinv: [owner, low ghost, high ghost];
    ghosts: [low, high]."""

    def __init__(self, xv, period, bounded: int, kinds, uinf=(0.0, 0.0, 0.0), gamma: float = 1.4, stream=None):
        super().__init__(xv, period, bounded, kinds, uinf, gamma, None, stream)

    def fill(self, q):
        self._fill_all([q])

    def residual(self, q, entropy_fix: float = 0.1, eps: float = 1e-6, viscous=None):
        return super().residual([q], entropy_fix, eps, viscous)[0]

    def steps(self, q, dt: float, nsteps: int, entropy_fix: float = 0.1, eps: float = 1e-6, viscous=None,
              work=None):
        super().steps([q], dt, nsteps, entropy_fix, eps, viscous, work)
        return q


class WcnsClosedDuct:
    """A curvilinear block periodic along one direction and closed across the
    other two (bounded = (d1, d2), d1 < d2; kinds[d] = (low, high) cfd_bc_kind
    of direction d): four face ghost blocks and four corner ghost blocks.
    xv: vertices with n_d + 1 planes along each bounded direction and the n_t
    upper corners along the periodic one (a CUDA tensor).  Blocks: 0 owner;
    1, 2 the low and high ghost blocks across d1; 3, 4 across d2; 5 .. 8 the
    corners (d1 side, d2 side) = (lo, lo), (lo, hi), (hi, lo), (hi, hi).  The
    corners are filled from the d1 ghost blocks after those (sweep order)."""

    def __init__(self, xv, period, bounded, kinds, uinf=(0.0, 0.0, 0.0), gamma: float = 1.4, stream=None):
        import torch
        self.torch = torch
        self.stream = stream
        d1, d2 = sorted(int(d) for d in bounded)
        self.d1, self.d2, self.uinf, self.gamma = d1, d2, tuple(uinf), float(gamma)
        self.kinds = {d1: tuple(kinds[d1]), d2: tuple(kinds[d2])}
        n = [int(xv.shape[3]), int(xv.shape[2]), int(xv.shape[1])]
        n[d1] -= 1
        n[d2] -= 1
        self.n = tuple(n)
        e = [n[d] + 1 + 2 * WCNS5_XLAYERS if d in (d1, d2) else n[d] + 5 for d in range(3)]
        xe = torch.empty((3, e[2], e[1], e[0]), dtype=torch.float64, device=xv.device)
        per = (C.c_double * 9)(*[float(v) for row in period for v in row])
        _check(lib().cfd_wcns5_extend_vertices_mask(_ptr(xv), (C.c_int32 * 3)(*n), (1 << d1) | (1 << d2), per,
                                                    _ptr(xe), _stream_handle(torch, stream)))
        G = WCNS5_GHOST
        spans = {d: {"own": (0, n[d]), "lo": (-G, G), "hi": (n[d], G)} for d in (d1, d2)}
        order = [("own", "own"), ("lo", "own"), ("hi", "own"), ("own", "lo"), ("own", "hi"),
                 ("lo", "lo"), ("lo", "hi"), ("hi", "lo"), ("hi", "hi")]
        org = [WCNS5_XLAYERS + 1 if d in (d1, d2) else 3 for d in range(3)]
        self.dims, self.S, self.jinv = [], [], []
        for w1, w2 in order:
            ext, sl = list(n), []
            ext[d1], ext[d2] = spans[d1][w1][1], spans[d2][w2][1]
            self.dims.append(tuple(ext))
            for a in (2, 1, 0):
                st = spans[d1][w1][0] if a == d1 else spans[d2][w2][0] if a == d2 else 0
                sl.append(slice(org[a] - 3 + st, org[a] - 3 + st + ext[a] + 5))
            S, J = wcns5_metrics_ext(xe[(slice(None),) + tuple(sl)].contiguous(), stream)
            self.S.append(S)
            self.jinv.append(J)
        idx = {w: b for b, w in enumerate(order)}
        nxt = {"lo": "own", "own": "hi", "hi": "lo"}
        self.nbr = [[b] * 6 for b in range(9)]
        for b, (w1, w2) in enumerate(order):
            up1, up2 = idx[(nxt[w1], w2)], idx[(w1, nxt[w2])]
            self.nbr[b][2 * d1 + 1], self.nbr[up1][2 * d1] = up1, b
            self.nbr[b][2 * d2 + 1], self.nbr[up2][2 * d2] = up2, b
        self.ghosts = [torch.zeros((5, m[2], m[1], m[0]), dtype=torch.float64, device=xv.device)
                       for m in self.dims[1:]]
        # (owner, low ghost, high ghost, direction), in fill order
        self.fills = [(0, 1, 2, d1), (0, 3, 4, d2), (1, 5, 6, d2), (2, 7, 8, d2)]

    def _all(self, q):
        return [q] + self.ghosts

    def fill(self, q):
        allq = self._all(q)
        for o, lo, hi, d in self.fills:
            wcns5_fill_ghost_blocks(allq[o], allq[lo], allq[hi], self.S[o], self.S[lo], d, self.kinds[d], self.uinf,
                                    self.gamma, self.stream)

    def residual(self, q, entropy_fix: float = 0.1, eps: float = 1e-6, viscous=None):
        """R of the owner (dQ/dt = -R); viscous = (prandtl, mu_inf, s_star)."""
        self.fill(q)
        allq = self._all(q)
        rs = wcns5_euler_residual_blocks(allq, self.S, self.jinv, self.nbr, self.gamma, entropy_fix, eps,
                                         stream=self.stream)
        if viscous is not None:
            c4_viscous_add_blocks(allq, rs, self.S, self.jinv, self.nbr, self.gamma, *viscous, stream=self.stream)
        return rs[0]

    def steps(self, q, dt: float, nsteps: int, entropy_fix: float = 0.1, eps: float = 1e-6, viscous=None,
              work=None):
        """nsteps RK3 steps in place on q (cfd_wcns5_steps_blocks_closed with the four fills)."""
        torch = self.torch
        allq = self._all(q)
        dims = (C.c_int32 * 27)(*[v for m in self.dims for v in m])
        nbt = (C.c_int32 * 54)(*[v for row in self.nbr for v in row])
        nbytes = C.c_size_t()
        _check(lib().cfd_wcns5_ns_blocks_work_bytes(9, dims, nbt, C.byref(nbytes)))
        if work is None or work.numel() * work.element_size() < nbytes.value:
            work = _scratch(torch, nbytes.value, q.device, self.stream)
        cls = (WcnsClosure * 4)(*[WcnsClosure(o, lo, hi, d, (C.c_int32 * 2)(*self.kinds[d]),
                                              (C.c_double * 3)(*self.uinf)) for o, lo, hi, d in self.fills])
        pr, mu, ss = viscous if viscous is not None else (0.72, 0.0, 110.4 / 288.15)
        ptrs = lambda ts: (C.c_void_p * 9)(*[_ptr(t) for t in ts])   # noqa: E731
        _check(lib().cfd_wcns5_steps_blocks_closed(9, dims, nbt, ptrs(allq), ptrs(self.S), ptrs(self.jinv), cls, 4,
                                                   1 if viscous is not None else 0, _ptr(work), nbytes.value,
                                                   self.gamma, float(entropy_fix), float(eps), float(pr), float(mu),
                                                   float(ss), float(dt), int(nsteps),
                                                   _stream_handle(torch, self.stream)))
        return q


def _on_device(torch, x, device):
    """A contiguous FP64 device tensor of a NumPy array or a tensor (a device
    tensor already in place is used as it is)."""
    if torch.is_tensor(x):
        return x.to(device=device, dtype=torch.float64).contiguous()
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float64)).to(device)


class Solver:
    """One context over one GPU's share of blocks.

    ``q`` is the caller-visible state arena (torch float64 on the device);
    ``views()`` gives per-block padded views [5, nk+2g, nj+2g, ni+2g].
    """

    def __init__(self, case, device: str = "cuda:0", tuning: Optional[dict] = None, stream=None):
        import torch
        self.torch = torch
        self.case = case
        self.device = torch.device(device)
        self.stream = stream
        L = lib()
        self.dims = list(case.dims)
        self.offsets, self.strides, self.arena_elems = layout(self.dims)
        self._pp = to_params(case.params)
        self._dims = to_dims(self.dims)
        ws = C.c_size_t()
        _check(L.cfd_workspace_size(C.byref(self._pp), len(self.dims), self._dims, C.byref(ws)))
        self.ws_bytes = int(ws.value)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
            self.q = torch.full((self.arena_elems,), float("nan"), dtype=torch.float64, device=self.device)
            nodes = [_on_device(torch, x, self.device) for x in case.nodes]
            nptrs = (C.c_void_p * len(nodes))(*[t.data_ptr() for t in nodes])
            conns = to_conns(case.conns)
            bcs = to_bcs(case.bcs)
            ctx = C.c_void_p()
            st = L.cfd_create_blocks(C.byref(self._pp), len(self.dims), self._dims, nptrs, len(case.conns),
                                     conns, len(case.bcs), bcs, _ptr(self.workspace),
                                     C.c_size_t(self.ws_bytes), self._s(), C.byref(ctx))
            _check(st)
            self.ctx = ctx
            del nodes
        if tuning:
            self.set_tuning(**tuning)
        self.set_state(case.q0)

    # ------------------------------------------------------------ plumbing
    def _s(self):
        return _stream_handle(self.torch, self.stream)

    def close(self):
        if getattr(self, "ctx", None):
            lib().cfd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tuning(self, kernel=None, tile_j=None, tile_k=None, use_graph=None, order=None):
        t = Tuning()
        _check(lib().cfd_get_tuning(self.ctx, C.byref(t)), self.ctx)
        for name, v in (("kernel", kernel), ("tile_j", tile_j), ("tile_k", tile_k), ("use_graph", use_graph),
                        ("order", order)):
            if v is not None:
                setattr(t, name, int(v))
        _check(lib().cfd_set_tuning(self.ctx, C.byref(t)), self.ctx)

    def get_tuning(self) -> dict:
        t = Tuning()
        _check(lib().cfd_get_tuning(self.ctx, C.byref(t)), self.ctx)
        return {n: getattr(t, n) for n, _ in Tuning._fields_}

    def views(self, arena=None):
        arena = self.q if arena is None else arena
        out = []
        for b, (ni, nj, nk) in enumerate(self.dims):
            sv, sk, sj, si = self.strides[b]
            out.append(arena.as_strided((5, nk + 2 * NG, nj + 2 * NG, ni + 2 * NG), (sv, sk, sj, si),
                                        self.offsets[b]))
        return out

    def interior_views(self, arena=None):
        return [v[:, NG:-NG, NG:-NG, NG:-NG] for v in self.views(arena)]

    def new_arena(self, fill=float("nan")):
        return self.torch.full((self.arena_elems,), fill, dtype=self.torch.float64, device=self.device)

    def set_state(self, q0: Sequence[np.ndarray], arena=None):
        arena = self.q if arena is None else arena
        for v, q in zip(self.interior_views(arena), q0):
            v.copy_(_on_device(self.torch, q, self.device))

    def state(self, arena=None) -> List[np.ndarray]:
        self.torch.cuda.synchronize(self.device)
        return [v.cpu().numpy().copy() for v in self.interior_views(arena)]

    # ------------------------------------------------------------ library calls
    def fill_ghosts(self, arena=None):
        arena = self.q if arena is None else arena
        _check(lib().cfd_fill_ghosts(self.ctx, _ptr(arena), self._s()), self.ctx)

    def residual(self, arena=None, fill=True):
        arena = self.q if arena is None else arena
        if fill:
            self.fill_ghosts(arena)
        r = self.new_arena()
        _check(lib().cfd_residual(self.ctx, _ptr(arena), _ptr(r), self._s()), self.ctx)
        return r

    def step(self, nsteps: int = 1, hist: bool = True, arena=None):
        arena = self.q if arena is None else arena
        h = None
        if hist and nsteps > 0:
            h = self.torch.zeros((nsteps, 12), dtype=self.torch.float64, device=self.device)
        _check(lib().cfd_step(self.ctx, _ptr(arena), int(nsteps), _ptr(h) if h is not None else None,
                              self._s()), self.ctx)
        return h

    def step_implicit(self, nsteps: int = 1, sweeps: int = 8, cfl: float = 20.0, hist: bool = True, arena=None):
        """nsteps implicit steps (cfd_step_implicit: backward Euler, frozen
        flux-split Jacobian, `sweeps` point-Jacobi sweeps, CFL step at `cfl`);
        returns the history [nsteps, 12] (device) or None."""
        arena = self.q if arena is None else arena
        torch = self.torch
        if getattr(self, "_impl_work", None) is None:
            nb = C.c_size_t()
            _check(lib().cfd_implicit_work_size(self.ctx, C.byref(nb)), self.ctx)
            self._impl_work = torch.empty(int(nb.value) + 256, dtype=torch.uint8, device=self.device)
        w = self._impl_work
        base = w.data_ptr()
        off = (-base) % 256
        h = None
        if hist and nsteps > 0:
            h = torch.zeros((nsteps, 12), dtype=torch.float64, device=self.device)
        _check(lib().cfd_step_implicit(self.ctx, _ptr(arena), int(nsteps), int(sweeps), float(cfl),
                                       C.c_void_p(base + off), C.c_size_t(w.numel() - off),
                                       _ptr(h) if h is not None else None, self._s()), self.ctx)
        return h

    def time_step(self, arena=None) -> float:
        arena = self.q if arena is None else arena
        d = self.torch.zeros(1, dtype=self.torch.float64, device=self.device)
        _check(lib().cfd_time_step(self.ctx, _ptr(arena), _ptr(d), self._s()), self.ctx)
        self.torch.cuda.synchronize(self.device)
        return float(d.item())

    def set_profiling(self, on: bool):
        _check(lib().cfd_set_profiling(self.ctx, 1 if on else 0), self.ctx)

    def profile_read(self) -> dict:
        """Per kernel class: launches, total/min/max ms (and mean) since the last read."""
        out = (C.c_double * 16)()
        _check(lib().cfd_profile_read(self.ctx, out), self.ctx)
        res = {}
        for k, name in enumerate(("stage", "ghost", "dt", "norms")):
            n, tot, mn, mx = out[4 * k:4 * k + 4]
            res[name] = {"launches": int(n), "total_ms": tot, "min_ms": mn, "max_ms": mx,
                         "mean_ms": tot / n if n else 0.0}
        return res

    def metrics(self, blk: int) -> np.ndarray:
        """Block blk's metrics [10, nk+2g, nj+2g, ni+2g] (S_i, S_j, S_k, V)."""
        ni, nj, nk = self.dims[blk]
        out = self.torch.empty((10, nk + 2 * NG, nj + 2 * NG, ni + 2 * NG), dtype=self.torch.float64,
                               device=self.device)
        _check(lib().cfd_copy_metrics(self.ctx, int(blk), _ptr(out), self._s()), self.ctx)
        self.torch.cuda.synchronize(self.device)
        return out.cpu().numpy()

    def norms(self, arena=None, r=None, check=True) -> np.ndarray:
        arena = self.q if arena is None else arena
        out = (C.c_double * 12)()
        st = lib().cfd_norms(self.ctx, _ptr(arena), _ptr(r) if r is not None else None, out, CFD_NORMS_HOST,
                             self._s())
        if st != CFD_OK and not (st == -4 and not check):
            _check(st, self.ctx)
        return np.array(out[:])

    # ------------------------------------------------------------ warm start
    def mlp_features(self, cond):
        """Features x[ncells][5] of every interior cell; cond [nblk][2] (Mach, bump height)."""
        torch = self.torch
        c = torch.as_tensor(np.asarray(cond, dtype=np.float64).reshape(-1, 2), device=self.device)
        x = torch.empty((self.case.ncells, 5), dtype=torch.float32, device=self.device)
        _check(lib().cfd_mlp_features(self.ctx, _ptr(c), _ptr(x), self._s()), self.ctx)
        return x

    def mlp_targets(self, cond, arena=None):
        arena = self.q if arena is None else arena
        torch = self.torch
        c = torch.as_tensor(np.asarray(cond, dtype=np.float64).reshape(-1, 2), device=self.device)
        t = torch.empty((self.case.ncells, 5), dtype=torch.float32, device=self.device)
        _check(lib().cfd_mlp_targets(self.ctx, _ptr(arena), _ptr(c), _ptr(t), self._s()), self.ctx)
        return t

    def mlp_to_state(self, y, cond, arena=None):
        arena = self.q if arena is None else arena
        c = self.torch.as_tensor(np.asarray(cond, dtype=np.float64).reshape(-1, 2), device=self.device)
        _check(lib().cfd_mlp_to_state(self.ctx, _ptr(y), _ptr(c), _ptr(arena), self._s()), self.ctx)


# ---------------------------------------------------------------------- MLP

def mlp_layout(d_in, d_hidden, n_hidden, d_out):
    """[(woff, N, K, boff)] of the padded parameter layout (see include/cfd.h)."""
    out, off = [], 0
    for l in range(n_hidden + 1):
        K = 16 if l == 0 else d_hidden
        N = 16 if l == n_hidden else d_hidden
        out.append((off, N, K, off + N * K))
        off += N * K + N
    return out, off


def pack_params(params, d_in, d_hidden, n_hidden, d_out):
    """Unpadded [(W [out, in], b)] -> padded flat float32 vector."""
    lay, total = mlp_layout(d_in, d_hidden, n_hidden, d_out)
    flat = np.zeros(total, dtype=np.float32)
    for (woff, N, K, boff), (W, b) in zip(lay, params):
        Wp = np.zeros((N, K), dtype=np.float32)
        Wp[:W.shape[0], :W.shape[1]] = W
        flat[woff:woff + N * K] = Wp.ravel()
        bp = np.zeros(N, dtype=np.float32)
        bp[:b.shape[0]] = b
        flat[boff:boff + N] = bp
    return flat


def unpack_params(flat, d_in, d_hidden, n_hidden, d_out):
    lay, _ = mlp_layout(d_in, d_hidden, n_hidden, d_out)
    sizes = [d_in] + [d_hidden] * n_hidden + [d_out]
    out = []
    for l, (woff, N, K, boff) in enumerate(lay):
        W = np.asarray(flat[woff:woff + N * K], dtype=np.float64).reshape(N, K)[:sizes[l + 1], :sizes[l]]
        b = np.asarray(flat[boff:boff + N], dtype=np.float64)[:sizes[l + 1]]
        out.append((W.copy(), b.copy()))
    return out


class Mlp:
    """Device-resident warm-start network: BF16 weights for inference, FP32
    master weights, Adam moments and gradients for training."""

    def __init__(self, params, d_in=5, d_hidden=128, n_hidden=4, d_out=5, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.stream = stream
        self.desc = MlpDesc(d_in, d_hidden, n_hidden, d_out, 1)
        self.dims = (d_in, d_hidden, n_hidden, d_out)
        npar = C.c_int64()
        cpp = C.c_int64()
        _check(lib().cfd_mlp_sizes(C.byref(self.desc), 0, C.byref(npar), C.byref(cpp), None))
        self.nparam, self.cache_per_point = int(npar.value), int(cpp.value)
        flat = pack_params(params, *self.dims)
        assert flat.size == self.nparam
        self.master = torch.from_numpy(flat).to(self.device)
        self.bf16 = torch.empty(self.nparam, dtype=torch.int16, device=self.device)
        self.m = torch.zeros_like(self.master)
        self.v = torch.zeros_like(self.master)
        self.grad = torch.zeros_like(self.master)
        self.t = 0
        self._work = None
        _check(lib().cfd_mlp_to_bf16(C.byref(self.desc), _ptr(self.master), _ptr(self.bf16), self._s()))

    def _s(self):
        return _stream_handle(self.torch, self.stream)

    def params(self):
        return unpack_params(self.master.cpu().numpy(), *self.dims)

    def bf16_params(self):
        """The BF16 weights as float64 (unpadded)."""
        raw = self.bf16.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
        return unpack_params(raw.view(np.float32), *self.dims)

    def workspace(self, n):
        ws = C.c_size_t()
        _check(lib().cfd_mlp_sizes(C.byref(self.desc), int(n), None, None, C.byref(ws)))
        if self._work is None or self._work.numel() < ws.value:
            self._work = self.torch.empty(int(ws.value), dtype=self.torch.uint8, device=self.device)
        return self._work, int(ws.value)

    def forward(self, x, idx=None, n=None, cache=False):
        torch = self.torch
        n = int(x.shape[0] if idx is None else idx.shape[0]) if n is None else n
        y = torch.empty((n, self.dims[3]), dtype=torch.float32, device=self.device)
        cb = torch.empty((n, self.cache_per_point), dtype=torch.float32, device=self.device) if cache else None
        _check(lib().cfd_mlp_forward(C.byref(self.desc), _ptr(self.bf16), _ptr(x),
                                     _ptr(idx) if idx is not None else None, n, _ptr(y),
                                     _ptr(cb) if cb is not None else None, self._s()))
        return (y, cb) if cache else y

    def mse(self, y, t, idx=None):
        torch = self.torch
        n = y.shape[0]
        dy = torch.empty_like(y)
        loss = torch.zeros(1, dtype=torch.float64, device=self.device)
        w, wb = self.workspace(n)
        _check(lib().cfd_mlp_mse(C.byref(self.desc), _ptr(y), _ptr(t), _ptr(idx) if idx is not None else None, n,
                                 _ptr(dy), _ptr(loss), _ptr(w), wb, self._s()))
        return loss, dy

    def backward(self, cache, dy):
        n = dy.shape[0]
        w, wb = self.workspace(n)
        _check(lib().cfd_mlp_backward(C.byref(self.desc), _ptr(self.bf16), _ptr(cache), _ptr(dy), n,
                                      _ptr(self.grad), _ptr(w), wb, self._s()))
        return self.grad

    def adam(self, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.t += 1
        _check(lib().cfd_mlp_adam(C.byref(self.desc), _ptr(self.master), _ptr(self.m), _ptr(self.v),
                                  _ptr(self.grad), _ptr(self.bf16), lr, b1, b2, eps, self.t, self._s()))

    def train_step(self, x, t, idx, lr=1e-3):
        """One minibatch: forward (with cache), MSE, backward, Adam; returns the loss tensor."""
        y, cache = self.forward(x, idx=idx, cache=True)
        loss, dy = self.mse(y, t, idx)
        self.backward(cache, dy)
        self.adam(lr)
        return loss
