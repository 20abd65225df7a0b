"""Python binding of ``libps.so`` (the C ABI declared in ``include/ps.h``).

Argument marshalling only: every step of a solve runs in the library's HIP
kernels.  The ``ps_*`` functions mirror the C entry points one to one and
raise :class:`PSError` on a non-zero status; :class:`Solver` wraps a plan
with a torch-allocated workspace for convenience.  torch supplies device
memory and streams and is imported before the library is loaded so that both
use the same HIP runtime instance.

If ``libps.so`` is missing the import of this module's functions fails with
an error: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, List, Optional, Sequence

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libps.so")

PS_OK = 0
PS_ERR_INVALID = -1
PS_ERR_UNSUPPORTED = -2
PS_ERR_NOT_READY = -3
PS_ERR_DEVICE = -4
PS_ERR_CAPTURE = -5

PS_F64 = 0
PS_F32 = 1
PS_F32_SPLIT = 2
PS_F64_PLAIN = 3
PS_F32_PLAIN = 4

PRECISIONS = {"f64": PS_F64, "f32": PS_F32, "f32_split": PS_F32_SPLIT,
              "f64_plain": PS_F64_PLAIN, "f32_plain": PS_F32_PLAIN}

# N = 8 m, m <= 64 with no prime factor above 5 (P = 2N = 2^a 3^b 5^c, a >= 4)
SUPPORTED_N = (8, 16, 24, 32, 40, 48, 64, 72, 80, 96, 120, 128, 144, 160, 192, 200, 216, 240, 256, 288, 320, 360,
               384, 400, 432, 480, 512)

EXPORTS = ("ps_plan_create", "ps_plan_workspace_bytes", "ps_plan_query", "ps_green_build", "ps_solve",
           "ps_solve_batched", "ps_plan_destroy", "ps_status_str", "ps_last_error", "ps_debug_pass",
           "ps_plan_set_variant", "ps_autotune", "ps_host_stage_bytes", "ps_solve_host", "ps_plan_set_spacing",
           "ps_stream_copy", "ps_solve_static", "ps_plan_create_box")


class PSError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: status {status}: {detail}")
        self.status = status


class PlanInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int), ("p", ctypes.c_int), ("h", ctypes.c_int), ("precision", ctypes.c_int),
                ("dx", ctypes.c_double), ("workspace_bytes", ctypes.c_size_t), ("ghat_bytes", ctypes.c_size_t),
                ("ready", ctypes.c_int), ("radices", ctypes.c_int * 8),
                ("t1_offset", ctypes.c_size_t), ("t2_offset", ctypes.c_size_t), ("t3_offset", ctypes.c_size_t),
                ("variant", ctypes.c_int * 5),
                ("split_terms", ctypes.c_int), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
                ("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int), ("z_tile", ctypes.c_int)]


_lib: Optional[ctypes.CDLL] = None


def load() -> ctypes.CDLL:
    """Load ``libps.so`` (after torch, so both share one HIP runtime)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2409_02294_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i, d, sz = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t
    sig = {
        "ps_plan_create": ([ctypes.POINTER(vp), i, d, i, ctypes.c_char_p], i),
        "ps_plan_create_box": ([ctypes.POINTER(vp), i, i, i, d, d, d, i, ctypes.c_char_p], i),
        "ps_plan_workspace_bytes": ([vp, ctypes.POINTER(sz)], i),
        "ps_plan_query": ([vp, ctypes.POINTER(PlanInfo)], i),
        "ps_green_build": ([vp, vp, d, d, vp], i),
        "ps_solve": ([vp, vp, vp, vp], i),
        "ps_solve_batched": ([ctypes.POINTER(vp), i, ctypes.POINTER(vp), ctypes.POINTER(vp), vp], i),
        "ps_host_stage_bytes": ([vp, ctypes.POINTER(sz)], i),
        "ps_solve_host": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), i, vp, sz, vp], i),
        "ps_plan_destroy": ([vp], None),
        "ps_status_str": ([i], ctypes.c_char_p),
        "ps_last_error": ([], ctypes.c_char_p),
        "ps_debug_pass": ([vp, i, vp, vp, vp], i),
        "ps_plan_set_variant": ([vp, i, i], i),
        "ps_plan_set_spacing": ([vp, ctypes.c_double, ctypes.c_double], i),
        "ps_autotune": ([vp, vp, ctypes.c_char_p], i),
        "ps_stream_copy": ([vp, vp, sz, vp], i),
        "ps_solve_static": ([vp, vp, vp, vp], i),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def _check(rc: int, where: str) -> None:
    if rc != PS_OK:
        lib = load()
        raise PSError(rc, where, lib.ps_last_error().decode())


def ps_status_str(status: int) -> str:
    return load().ps_status_str(status).decode()


def ps_last_error() -> str:
    return load().ps_last_error().decode()


def ps_plan_create(n: int, dx: float, precision: int, tune_cache: Optional[str] = None) -> int:
    h = ctypes.c_void_p()
    tc = tune_cache.encode() if tune_cache else None
    _check(load().ps_plan_create(ctypes.byref(h), int(n), float(dx), int(precision), tc), "ps_plan_create")
    return h.value


def ps_plan_create_box(nx: int, ny: int, nz: int, dx: float, dy: float, dz: float, precision: int,
                       tune_cache: Optional[str] = None) -> int:
    h = ctypes.c_void_p()
    tc = tune_cache.encode() if tune_cache else None
    _check(load().ps_plan_create_box(ctypes.byref(h), int(nx), int(ny), int(nz), float(dx), float(dy), float(dz),
                                     int(precision), tc), "ps_plan_create_box")
    return h.value


def ps_plan_workspace_bytes(plan: int) -> int:
    b = ctypes.c_size_t()
    _check(load().ps_plan_workspace_bytes(plan, ctypes.byref(b)), "ps_plan_workspace_bytes")
    return b.value


def ps_plan_query(plan: int) -> Dict:
    info = PlanInfo()
    _check(load().ps_plan_query(plan, ctypes.byref(info)), "ps_plan_query")
    rad = [r for r in info.radices if r]
    return dict(n=info.n, p=info.p, h=info.h, precision=info.precision, dx=info.dx,
                workspace_bytes=info.workspace_bytes, ghat_bytes=info.ghat_bytes, ready=bool(info.ready),
                radices=rad, t1_offset=info.t1_offset, t2_offset=info.t2_offset, t3_offset=info.t3_offset, variant=list(info.variant), split_terms=info.split_terms,
                dy=info.dy, dz=info.dz, nx=info.nx, ny=info.ny, nz=info.nz, z_tile=info.z_tile)


def ps_green_build(plan: int, workspace: int, G: float, self_coeff: float, stream: int) -> None:
    _check(load().ps_green_build(plan, workspace, float(G), float(self_coeff), stream), "ps_green_build")


def ps_solve(plan: int, rho: int, phi: int, stream: int) -> None:
    _check(load().ps_solve(plan, rho, phi, stream), "ps_solve")


def ps_solve_batched(plans: Sequence[int], rho: Sequence[int], phi: Sequence[int], stream: int) -> None:
    n = len(plans)
    if len(rho) != n or len(phi) != n:
        raise ValueError("plans, rho and phi must have equal length")
    arr = ctypes.c_void_p * max(n, 1)
    _check(load().ps_solve_batched(arr(*plans), n, arr(*rho), arr(*phi), stream), "ps_solve_batched")


def ps_host_stage_bytes(plan: int) -> int:
    v = ctypes.c_size_t()
    _check(load().ps_host_stage_bytes(plan, ctypes.byref(v)), "ps_host_stage_bytes")
    return v.value


def ps_solve_host(plan: int, rho: Sequence[int], phi: Sequence[int], stage: int, stage_bytes: int,
                  stream: int) -> None:
    n = len(rho)
    if len(phi) != n:
        raise ValueError("rho and phi must have equal length")
    arr = ctypes.c_void_p * max(n, 1)
    _check(load().ps_solve_host(plan, arr(*rho), arr(*phi), n, stage, stage_bytes, stream), "ps_solve_host")


def ps_plan_destroy(plan: int) -> None:
    if plan:
        load().ps_plan_destroy(plan)


def ps_debug_pass(plan: int, pass_id: int, d_in: int, d_out: int, stream: int) -> None:
    _check(load().ps_debug_pass(plan, int(pass_id), d_in, d_out, stream), "ps_debug_pass")


def ps_plan_set_variant(plan: int, pass_id: int, variant: int) -> None:
    _check(load().ps_plan_set_variant(plan, int(pass_id), int(variant)), "ps_plan_set_variant")


def ps_plan_set_spacing(plan: int, dy: float, dz: float) -> None:
    _check(load().ps_plan_set_spacing(plan, float(dy), float(dz)), "ps_plan_set_spacing")


def ps_solve_static(plan: int, rho: int, phi: int, stream: int) -> None:
    _check(load().ps_solve_static(plan, rho, phi, stream), "ps_solve_static")


def ps_stream_copy(src: int, dst: int, nbytes: int, stream: int) -> None:
    _check(load().ps_stream_copy(src, dst, int(nbytes), stream), "ps_stream_copy")


def ps_autotune(plan: int, stream: int, cache_path: Optional[str] = None) -> None:
    cp = cache_path.encode() if cache_path else None
    _check(load().ps_autotune(plan, stream, cp), "ps_autotune")


# ---------------------------------------------------------------------------
# torch convenience wrapper
# ---------------------------------------------------------------------------

class Solver:
    """A plan plus its torch-allocated workspace on one device.

    ``Solver(n, dx, "f32")(rho)`` returns the potential of the ``(n, n, n)``
    density tensor ``rho`` (float64 for f64 precisions, float32 otherwise)
    as a new tensor, enqueued on torch's current stream.  ``n`` may also be a
    box ``(nx, ny, nz)`` (tensors of shape ``(nz, ny, nx)``, a plan from
    ps_plan_create_box), with ``spacing=(dy, dz)`` as for cubes.
    """

    def __init__(self, n: int, dx: Optional[float] = None, precision="f32", G: float = 1.0,
                 self_coeff: float = 2.38, device=None, tune_cache: Optional[str] = None,
                 spacing: Optional[tuple] = None):
        import torch
        self.torch = torch
        dims = tuple(int(v) for v in n) if isinstance(n, (tuple, list)) else (int(n),) * 3
        self.n = dims[0]
        self.shape = (dims[2], dims[1], dims[0])  # [z][y][x]
        self.dx = float(dx) if dx is not None else 1.0 / self.n
        self.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        self.dtype = torch.float64 if self.precision in (PS_F64, PS_F64_PLAIN) else torch.float32
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if dims[0] == dims[1] == dims[2]:
            self.plan = ps_plan_create(self.n, self.dx, self.precision, tune_cache)
            if spacing is not None:  # (dy, dz): cells of spacings dx, dy, dz
                ps_plan_set_spacing(self.plan, spacing[0], spacing[1])
        else:
            dy, dz = spacing if spacing is not None else (self.dx, self.dx)
            self.plan = ps_plan_create_box(dims[0], dims[1], dims[2], self.dx, dy, dz, self.precision, tune_cache)
        nbytes = ps_plan_workspace_bytes(self.plan)
        with torch.cuda.device(self.device):
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            stream = torch.cuda.current_stream(self.device).cuda_stream
            ps_green_build(self.plan, self.workspace.data_ptr(), G, self_coeff, stream)

    def solve_host(self, rhos, outs=None, stage=None):
        """Solves of host-resident densities (CPU tensors, pinned for overlap),
        staged through device memory (ps_solve_host); returns the host outputs
        once `stream` has them."""
        torch = self.torch
        if outs is None:
            outs = [torch.empty_like(r) for r in rhos]
        for t in list(rhos) + list(outs):
            if t.device.type != "cpu" or t.dtype != self.dtype or tuple(t.shape) != self.shape or not t.is_contiguous():
                raise ValueError(f"host arrays must be contiguous {self.dtype} CPU tensors of shape {self.shape}")
        nbytes = ps_host_stage_bytes(self.plan)
        if stage is None:
            stage = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            stream = torch.cuda.current_stream(self.device)
            ps_solve_host(self.plan, [r.data_ptr() for r in rhos], [o.data_ptr() for o in outs], stage.data_ptr(),
                          stage.numel(), stream.cuda_stream)
            stream.synchronize()
        return outs

    def info(self) -> Dict:
        return ps_plan_query(self.plan)

    def _check_tensor(self, t, name):
        if t.device != self.device or t.dtype != self.dtype or tuple(t.shape) != self.shape or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of shape {self.shape} on {self.device}")

    def solve(self, rho, out=None):
        torch = self.torch
        self._check_tensor(rho, "rho")
        if out is None:
            out = torch.empty_like(rho)
        self._check_tensor(out, "out")
        stream = torch.cuda.current_stream(self.device).cuda_stream
        ps_solve(self.plan, rho.data_ptr(), out.data_ptr(), stream)
        return out

    __call__ = solve

    def close(self):
        if getattr(self, "plan", None):
            ps_plan_destroy(self.plan)
            self.plan = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batched(solvers: List[Solver], rhos, outs=None):
    """One batched solve (ps_solve_batched) over several solvers' densities."""
    import torch
    if outs is None:
        outs = [torch.empty_like(r) for r in rhos]
    for s, r, o in zip(solvers, rhos, outs):
        s._check_tensor(r, "rho")
        s._check_tensor(o, "out")
    stream = torch.cuda.current_stream(solvers[0].device).cuda_stream
    ps_solve_batched([s.plan for s in solvers], [r.data_ptr() for r in rhos], [o.data_ptr() for o in outs], stream)
    return outs
