"""Python binding of the C ABI in include/dg.h and include/dg_host.h.

Argument marshalling only: every computation happens in libdg.so (host setup
in C++, the right-hand side and time stepping in HIP kernels).  PyTorch is
used for device memory and streams.  If the library is missing the import
of this module fails; there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdg.so")

DG_OK, DG_EINVAL, DG_EMESH, DG_EHIP, DG_ENOMEM, DG_EUNSUPPORTED = 0, -1, -2, -3, -4, -5
DG_FP64, DG_FP32, DG_BF16X3, DG_F16X3, DG_BF16, DG_F16, DG_BF16X2, DG_F16X2 = range(8)
PRECISIONS = {"fp64": DG_FP64, "fp32": DG_FP32, "bf16x3": DG_BF16X3, "f16x3": DG_F16X3, "bf16": DG_BF16,
              "f16": DG_F16, "bf16x2": DG_BF16X2, "f16x2": DG_F16X2}

#: every symbol the public headers declare
EXPORTED = ("dg_setup_mesh", "dg_info_get", "dg_rhs", "dg_rk_step", "dg_pack", "dg_unpack", "dg_nodes",
            "dg_destroy", "dg_last_error", "dg_variant_count", "dg_variant_name", "dg_set_variant", "dg_time_rhs",
            "dg_setup_batch", "dg_batch_problem", "dg_rk_step_batch", "dg_destroy_batch", "dg_rk_step_noalloc", "dg_energy",
            "dg_system_compile", "dg_setup_system", "dg_set_tile_order",
            "dg_host_ref_nodes", "dg_host_ref_operators", "dg_host_mesh")


class DgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"dg status {status}: {msg}")
        self.status = status


DG_BC_CONDUCTING, DG_BC_MAGNETIC, DG_BC_ABSORBING = 0, 1, 2


class MeshDesc(C.Structure):
    _fields_ = [("N", C.c_int32), ("precision", C.c_int32), ("alpha", C.c_double),
                ("Nv", C.c_int64), ("VX", C.POINTER(C.c_double)),
                ("K", C.c_int64), ("EToV", C.POINTER(C.c_int32)),
                ("face_bc", C.POINTER(C.c_int8)), ("eps", C.POINTER(C.c_double)),
                ("mu", C.POINTER(C.c_double)), ("device", C.c_int32)]


class Info(C.Structure):
    _fields_ = [("N", C.c_int32), ("Np", C.c_int32), ("Nfp", C.c_int32), ("precision", C.c_int32),
                ("K", C.c_int64), ("field_stride", C.c_int64), ("state_elems", C.c_int64),
                ("elem_bytes", C.c_int32), ("tile_elems", C.c_int32), ("dt_cfl1", C.c_double),
                ("alpha", C.c_double), ("n_boundary_faces", C.c_int64), ("variant", C.c_int32),
                ("nfields", C.c_int32)]


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1211_0582_amd.build`")
    # PyTorch ships its own HIP runtime with the same SONAME as the system one.
    # Loading torch first makes libdg.so bind to that runtime, so the process
    # holds exactly one HIP runtime and device pointers/streams are shared.
    import torch  # noqa: F401
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    sig = {
        "dg_setup_mesh": (C.c_int, [C.POINTER(MeshDesc), C.POINTER(P)]),
        "dg_info_get": (C.c_int, [P, C.POINTER(Info)]),
        "dg_rhs": (C.c_int, [P, P, P, P]),
        "dg_rk_step": (C.c_int, [P, P, P, C.c_double, C.c_double, C.c_int32, P]),
        "dg_rk_step_noalloc": (C.c_int, [P, P, P, C.c_double, C.c_double, C.c_int32, P]),
        "dg_energy": (C.c_int, [P, P, P, P, P]),
        "dg_system_compile": (C.c_int, [C.c_char_p, C.c_int32, C.c_int32, C.c_int32, C.c_char_p, P, C.c_int64]),
        "dg_setup_system": (C.c_int, [C.POINTER(MeshDesc), C.c_char_p, C.c_int32, C.POINTER(P)]),
        "dg_pack": (C.c_int, [P, P, P, P]),
        "dg_unpack": (C.c_int, [P, P, P, P]),
        "dg_nodes": (C.c_int, [P, P]),
        "dg_destroy": (None, [P]),
        "dg_last_error": (C.c_char_p, []),
        "dg_variant_count": (C.c_int32, []),
        "dg_variant_name": (C.c_char_p, [C.c_int32]),
        "dg_set_variant": (C.c_int, [P, C.c_int32]),
        "dg_set_tile_order": (C.c_int, [P, C.c_int32]),
        "dg_time_rhs": (C.c_int, [P, P, P, C.c_int32, C.c_int32, P, C.POINTER(C.c_double)]),
        "dg_setup_batch": (C.c_int, [C.c_int32, C.POINTER(MeshDesc), C.POINTER(P)]),
        "dg_batch_problem": (C.c_int, [P, C.c_int32, C.POINTER(P)]),
        "dg_rk_step_batch": (C.c_int, [P, C.POINTER(P), C.POINTER(P), C.POINTER(C.c_double), C.c_int32, C.c_int32, P]),
        "dg_destroy_batch": (None, [P]),
        "dg_host_ref_nodes": (C.c_int, [C.c_int32, P, P, P]),
        "dg_host_ref_operators": (C.c_int, [C.c_int32, P, P, P, P, P, P]),
        "dg_host_mesh": (C.c_int, [C.c_int32, C.c_int64, P, C.c_int64, P, P, P, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def _check(status):
    if status != DG_OK:
        raise DgError(status, lib.dg_last_error().decode())


def _ptr(a):
    if a is None:
        return None
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()  # torch tensor


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def n_p(N):
    return (N + 1) * (N + 2) * (N + 3) // 6


def n_fp(N):
    return (N + 1) * (N + 2) // 2


# ---------------------------------------------------------------------------
# Host-side calls (no GPU needed)
# ---------------------------------------------------------------------------
def dg_host_ref_nodes(N):
    Np = n_p(N)
    r, s, t = (np.zeros(Np) for _ in range(3))
    _check(lib.dg_host_ref_nodes(N, _ptr(r), _ptr(s), _ptr(t)))
    return r, s, t


def dg_host_ref_operators(N):
    Np, Nfp = n_p(N), n_fp(N)
    Dr, Ds, Dt = (np.zeros((Np, Np)) for _ in range(3))
    LIFT = np.zeros((Np, 4 * Nfp))
    Fmask = np.zeros((4, Nfp), dtype=np.int32)
    Mf = np.zeros((4, Nfp, Nfp))
    _check(lib.dg_host_ref_operators(N, _ptr(Dr), _ptr(Ds), _ptr(Dt), _ptr(LIFT), _ptr(Fmask), _ptr(Mf)))
    return dict(Dr=Dr, Ds=Ds, Dt=Dt, LIFT=LIFT, Fmask=Fmask, Mf=Mf)


def _face_bc(face_bc, K):
    if face_bc is None:
        return None
    face_bc = np.ascontiguousarray(face_bc, dtype=np.int8)
    if face_bc.shape != (K, 4):
        raise ValueError(f"face_bc must have shape ({K}, 4)")
    return face_bc


def _per_element(v, K, name):
    if v is None:
        return None
    v = np.ascontiguousarray(np.broadcast_to(np.asarray(v, dtype=np.float64), (K,)))
    return v


def _cptr(a, ctype):
    return None if a is None else a.ctypes.data_as(C.POINTER(ctype))


def dg_host_mesh(N, VX, EToV, face_bc=None):
    VX = np.ascontiguousarray(VX, dtype=np.float64)
    EToV = np.ascontiguousarray(EToV, dtype=np.int32)
    K = EToV.shape[0]
    Nfp = n_fp(N)
    bc = _face_bc(face_bc, K)
    out = dict(metric=np.zeros((K, 9)), J=np.zeros(K), face=np.zeros((K, 4, 4)), sJ=np.zeros((K, 4)),
               vmapP=np.zeros((K, 4, Nfp), dtype=np.int64), conn=np.zeros((K, 4), dtype=np.int32))
    _check(lib.dg_host_mesh(N, VX.shape[0], _ptr(VX), K, _ptr(EToV), None if bc is None else _ptr(bc),
                            _ptr(out["metric"]), _ptr(out["J"]), _ptr(out["face"]), _ptr(out["sJ"]),
                            _ptr(out["vmapP"]), _ptr(out["conn"])))
    return out


# ---------------------------------------------------------------------------
# Device calls
# ---------------------------------------------------------------------------
def mesh_desc(N, VX, EToV, precision=DG_FP64, alpha=1.0, face_bc=None, eps=None, mu=None, device=-1):
    """(MeshDesc, keep-alive list of the host arrays it points into)."""
    VX = np.ascontiguousarray(VX, dtype=np.float64)
    EToV = np.ascontiguousarray(EToV, dtype=np.int32)
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    K = EToV.shape[0]
    bc = _face_bc(face_bc, K)
    ep = _per_element(eps, K, "eps")
    mu_ = _per_element(mu, K, "mu")
    d = MeshDesc(N, precision, alpha, VX.shape[0], _cptr(VX, C.c_double), K, _cptr(EToV, C.c_int32),
                 _cptr(bc, C.c_int8), _cptr(ep, C.c_double), _cptr(mu_, C.c_double), int(device))
    return d, [VX, EToV, bc, ep, mu_]


def dg_setup_mesh(N, VX, EToV, precision=DG_FP64, alpha=1.0, face_bc=None, eps=None, mu=None, device=-1):
    d, keep = mesh_desc(N, VX, EToV, precision, alpha, face_bc, eps, mu, device)
    h = C.c_void_p()
    _check(lib.dg_setup_mesh(C.byref(d), C.byref(h)))
    del keep
    return h


def dg_setup_system(N, VX, EToV, source, nfields, precision=DG_FP64, alpha=1.0, face_bc=None, device=-1):
    d, keep = mesh_desc(N, VX, EToV, precision, alpha, face_bc, None, None, device)
    h = C.c_void_p()
    _check(lib.dg_setup_system(C.byref(d), source.encode(), int(nfields), C.byref(h)))
    del keep
    return h


def dg_system_compile(source, nfields, N, precision=DG_FP64, arch="gfx950"):
    """Compiles a system's source with hipRTC (no device needed); returns the log."""
    if isinstance(precision, str):
        precision = PRECISIONS[precision]
    log = C.create_string_buffer(1 << 16)
    _check(lib.dg_system_compile(source.encode(), int(nfields), int(N), int(precision), arch.encode(), log, len(log)))
    return log.value.decode(errors="replace")


def dg_info_get(p):
    info = Info()
    _check(lib.dg_info_get(p, C.byref(info)))
    return info


def dg_rhs(p, u, rhs, stream=None):
    _check(lib.dg_rhs(p, _ptr(u), _ptr(rhs), _stream(stream)))


def dg_rk_step(p, u, res, t, dt, nsteps, stream=None):
    _check(lib.dg_rk_step(p, _ptr(u), _ptr(res), float(t), float(dt), int(nsteps), _stream(stream)))


def dg_rk_step_noalloc(p, u, res, t, dt, nsteps, stream=None):
    _check(lib.dg_rk_step_noalloc(p, _ptr(u), _ptr(res), float(t), float(dt), int(nsteps), _stream(stream)))


def dg_energy(p, u, ref, dev_out, stream=None):
    _check(lib.dg_energy(p, _ptr(u), _ptr(ref), _ptr(dev_out), _stream(stream)))


def dg_pack(p, host_u, dev_u, stream=None):
    host_u = np.ascontiguousarray(host_u, dtype=np.float64)
    _check(lib.dg_pack(p, _ptr(host_u), _ptr(dev_u), _stream(stream)))


def dg_unpack(p, dev_u, stream=None):
    info = dg_info_get(p)
    out = np.zeros((info.nfields, info.K, info.Np))
    _check(lib.dg_unpack(p, _ptr(dev_u), _ptr(out), _stream(stream)))
    return out


def dg_nodes(p):
    info = dg_info_get(p)
    xyz = np.zeros((info.K, info.Np, 3))
    _check(lib.dg_nodes(p, _ptr(xyz)))
    return xyz


def dg_destroy(p):
    lib.dg_destroy(p)


def dg_variant_count():
    return int(lib.dg_variant_count())


def dg_variant_name(v):
    n = lib.dg_variant_name(int(v))
    return None if n is None else n.decode()


def dg_time_rhs(p, u, rhs, warmup=3, reps=20, stream=None):
    ms = C.c_double()
    _check(lib.dg_time_rhs(p, _ptr(u), _ptr(rhs), int(warmup), int(reps), _stream(stream), C.byref(ms)))
    return ms.value


def variant_id(name):
    for v in range(dg_variant_count()):
        if dg_variant_name(v) == name:
            return v
    raise ValueError(f"unknown variant {name!r}")


def dg_set_variant(p, v):
    if isinstance(v, str):
        v = variant_id(v)
    _check(lib.dg_set_variant(p, int(v)))


# ---------------------------------------------------------------------------
# Convenience wrapper
# ---------------------------------------------------------------------------
class Problem:
    """Owns a dg_problem handle; allocates state arrays as torch tensors."""

    def __init__(self, N, VX, EToV, precision="fp64", alpha=1.0, tuned=False, face_bc=None, eps=None, mu=None,
                 device=-1):
        """tuned: apply the variant the autotuner cache holds for (N, precision, size).
        face_bc: (K, 4) boundary condition codes (DG_BC_*), eps / mu: per-element
        material (scalar or (K,)), device: HIP device ordinal (-1: current)."""
        self.handle = None
        self.handle = dg_setup_mesh(N, VX, EToV, precision, alpha, face_bc, eps, mu, device)
        self.info = dg_info_get(self.handle)
        if tuned:
            from . import autotune
            v = autotune.lookup(N, self.info.precision, self.info.K)
            if v is not None:
                self.set_variant(v)

    @property
    def torch_dtype(self):
        import torch
        return torch.float64 if self.info.precision == DG_FP64 else torch.float32

    def empty_state(self):
        import torch
        return torch.empty(self.info.state_elems, dtype=self.torch_dtype, device="cuda")

    def zeros_state(self):
        import torch
        return torch.zeros(self.info.state_elems, dtype=self.torch_dtype, device="cuda")

    def check_state(self, x, name="state"):
        """Device state arrays must be contiguous CUDA tensors of the problem's
        dtype with at least state_elems entries (the C ABI cannot see sizes)."""
        if not (getattr(x, "is_cuda", False) and x.is_contiguous() and x.dtype == self.torch_dtype
                and x.numel() >= self.info.state_elems):
            raise ValueError(f"{name}: need a contiguous cuda {self.torch_dtype} tensor with >= "
                             f"{self.info.state_elems} elements")
        return x

    def pack(self, host_u, dev_u=None, stream=None):
        dev_u = self.empty_state() if dev_u is None else self.check_state(dev_u, "dev_u")
        host_u = np.asarray(host_u, dtype=np.float64)
        shape = (self.info.nfields, self.info.K, self.info.Np)
        if host_u.shape != shape:
            raise ValueError(f"host_u must have shape {shape}")
        dg_pack(self.handle, host_u, dev_u, stream)
        return dev_u

    def unpack(self, dev_u, stream=None):
        return dg_unpack(self.handle, self.check_state(dev_u, "dev_u"), stream)

    def rhs(self, u, out, stream=None):
        dg_rhs(self.handle, self.check_state(u, "u"), self.check_state(out, "out"), stream)

    def rk_step(self, u, res, t, dt, nsteps=1, stream=None):
        dg_rk_step(self.handle, self.check_state(u, "u"), self.check_state(res, "res"), t, dt, nsteps, stream)

    def nodes(self):
        return dg_nodes(self.handle)

    def energy(self, u, ref=None, out=None, stream=None):
        """Discrete (material-weighted) energy of u - ref on the device; returns
        the one-element float64 device tensor it was written to."""
        import torch
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device="cuda")
        dg_energy(self.handle, self.check_state(u, "u"), None if ref is None else self.check_state(ref, "ref"),
                  out, stream)
        return out

    def error_norm(self, u, ref, stream=None):
        """L2 (mass-matrix) norm of u - ref, computed on the device (synchronises)."""
        return float(2.0 * self.energy(u, ref, stream=stream).item()) ** 0.5

    def set_tile_order(self, enable: bool):
        _check(lib.dg_set_tile_order(self.handle, int(bool(enable))))

    def set_variant(self, v):
        dg_set_variant(self.handle, v)
        self.info = dg_info_get(self.handle)

    @property
    def variant(self):
        return dg_variant_name(self.info.variant)

    def close(self):
        if self.handle:
            dg_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---------------------------------------------------------------------------
# Batches
# ---------------------------------------------------------------------------
BATCH_MODES = {"graph": 0, "grouped": 1, "per_problem": 2}


class _Borrowed(Problem):
    """Problem handle owned by a batch (never destroyed by itself)."""

    def __init__(self, handle):
        self.handle = handle
        self.info = dg_info_get(handle)

    def close(self):
        self.handle = None


class Batch:
    """n independent problems stepped together (dg_setup_batch)."""

    def __init__(self, meshes, precision="fp32", alpha=1.0):
        """meshes: list of (N, VX, EToV) or (N, VX, EToV, face_bc)."""
        self.handle = None
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        keep = []
        descs = (MeshDesc * len(meshes))()
        for i, mesh in enumerate(meshes):
            N, VX, EToV = mesh[:3]
            face_bc = mesh[3] if len(mesh) > 3 else None
            descs[i], k = mesh_desc(N, VX, EToV, precision, alpha, face_bc)
            keep += k
        h = C.c_void_p()
        _check(lib.dg_setup_batch(len(meshes), descs, C.byref(h)))
        self.handle = h
        self.problems = []
        for i in range(len(meshes)):
            ph = C.c_void_p()
            _check(lib.dg_batch_problem(h, i, C.byref(ph)))
            self.problems.append(_Borrowed(ph))

    def rk_step(self, us, ress, dts, nsteps=1, mode="graph", stream=None):
        n = len(self.problems)
        if not (len(us) == len(ress) == len(dts) == n):
            raise ValueError(f"need {n} state arrays, residuals and time steps")
        for p, u, r in zip(self.problems, us, ress):
            p.check_state(u, "u")
            p.check_state(r, "res")
        U = (C.c_void_p * n)(*[u.data_ptr() for u in us])
        R = (C.c_void_p * n)(*[r.data_ptr() for r in ress])
        Dt = (C.c_double * n)(*[float(d) for d in dts])
        _check(lib.dg_rk_step_batch(self.handle, U, R, Dt, int(nsteps), BATCH_MODES.get(mode, mode), _stream(stream)))

    def close(self):
        if self.handle:
            lib.dg_destroy_batch(self.handle)
            self.handle = None
            self.problems = []

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
