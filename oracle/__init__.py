"""FP64 CPU oracle for the free-space FFT-convolution potential solve.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product library never imports,
links or runs anything here, and nothing here imports the product library.

The arithmetic lives in ``oracle.c`` (plain C, IEEE double, OpenMP over
output cells and pencils); this module compiles it with gcc and wraps it with
ctypes.  Functions:

* :func:`direct_sum`        -- the definition, phi[i] = G dx^3 sum_j K(i-j) rho[j]
* :func:`direct_sum_cells`  -- the same at selected cells
* :func:`fft_conv`          -- the same via zero padding to 2N and full complex DFTs
* :func:`fft_conv_kernel`   -- as ``fft_conv`` with a caller-supplied padded kernel
* :func:`kernel_pad`, :func:`green_hat`, :func:`fft`, :func:`fft3`
* :func:`direct_sum3`, :func:`direct_sum_cells3`, :func:`fft_conv3`,
  :func:`kernel_pad3`, :func:`kernel_value3` -- the same on cells of spacings
  dx, dy, dz (x, y, z); :func:`cell_average_inv_r` -- the self-cell average
  of 1/|r| over such a cell
* :func:`direct_sum_box`, :func:`direct_sum_cells_box`, :func:`fft_conv_box`,
  :func:`kernel_pad_box`, :func:`fft3_box` -- boxes of nx x ny x nz cells
  (arrays [z][y][x]) with spacings dx, dy, dz, each axis padded to twice its
  own length

Kernel: K(d) = -1/(dx |d|) for d != 0, K(0) = -self_coeff/dx (default 2.38).
On dx x dy x dz cells: K(d) = -1/|(di dx, dj dy, dk dz)| and, unless the cell
is a cube, K(0) = -(self_coeff / (3 ln(2 + sqrt 3) - pi/2)) * cell_average_inv_r.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib: Optional[ctypes.CDLL] = None

SELF_COEFF = 2.38


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` next to it (gcc, -O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _bind(lib: ctypes.CDLL) -> ctypes.CDLL:
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    i, d = ctypes.c_int, ctypes.c_double
    sigs = {
        "or_set_threads": ([i], i),
        "or_get_threads": ([], i),
        "or_kernel_value": ([ctypes.c_long, ctypes.c_long, ctypes.c_long, d, d], d),
        "or_direct_sum": ([i, d, d, d, dp, dp], i),
        "or_direct_sum_cells": ([i, d, d, d, dp, i, ip, dp], i),
        "or_fft": ([i, dp, dp, i], i),
        "or_fft3": ([i, dp, i], i),
        "or_kernel_pad": ([i, d, d, dp], i),
        "or_green_hat": ([i, d, d, dp], i),
        "or_fft_conv_kernel": ([i, d, d, dp, dp, dp], i),
        "or_fft_conv": ([i, d, d, d, dp, dp], i),
        "or_cell_average_inv_r": ([d, d, d], d),
        "or_kernel_value3": ([ctypes.c_long, ctypes.c_long, ctypes.c_long, d, d, d, d], d),
        "or_direct_sum3": ([i, d, d, d, d, d, dp, dp], i),
        "or_direct_sum_cells3": ([i, d, d, d, d, d, dp, i, ip, dp], i),
        "or_kernel_pad3": ([i, d, d, d, d, dp], i),
        "or_fft_conv3": ([i, d, d, d, d, d, dp, dp], i),
        "or_direct_sum_box": ([i, i, i, d, d, d, d, d, dp, dp], i),
        "or_direct_sum_cells_box": ([i, i, i, d, d, d, d, d, dp, i, ip, dp], i),
        "or_fft3_box": ([i, i, i, dp, i], i),
        "or_kernel_pad_box": ([i, i, i, d, d, d, d, dp], i),
        "or_fft_conv_box": ([i, i, i, d, d, d, d, d, dp, dp], i),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


def _load() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build(force=True)
    _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc: int, what: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def _cube(rho: np.ndarray) -> np.ndarray:
    rho = np.ascontiguousarray(rho, dtype=np.float64)
    if rho.ndim != 3 or len(set(rho.shape)) != 1:
        raise ValueError("density must be a cubic [z][y][x] array")
    return rho


class Oracle:
    """The oracle's functions bound to one build of ``oracle.c``."""

    def __init__(self, lib: Optional[ctypes.CDLL] = None):
        self._l = lib

    @property
    def lib(self) -> ctypes.CDLL:
        return self._l if self._l is not None else _load()

    def set_threads(self, n: int) -> int:
        return self.lib.or_set_threads(int(n))

    def get_threads(self) -> int:
        return self.lib.or_get_threads()

    def kernel_value(self, di: int, dj: int, dk: int, dx: float, self_coeff: float = SELF_COEFF) -> float:
        return self.lib.or_kernel_value(int(di), int(dj), int(dk), float(dx), float(self_coeff))

    def direct_sum(self, rho: np.ndarray, dx: float, G: float = 1.0, self_coeff: float = SELF_COEFF) -> np.ndarray:
        rho = _cube(rho)
        phi = np.empty_like(rho)
        _check(self.lib.or_direct_sum(rho.shape[0], dx, G, self_coeff, _dp(rho), _dp(phi)), "direct_sum")
        return phi

    def direct_sum_cells(self, rho: np.ndarray, cells: Sequence[Sequence[int]], dx: float, G: float = 1.0,
                         self_coeff: float = SELF_COEFF) -> np.ndarray:
        rho = _cube(rho)
        c = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, 3))
        out = np.empty(c.shape[0], dtype=np.float64)
        rc = self.lib.or_direct_sum_cells(rho.shape[0], dx, G, self_coeff, _dp(rho), int(c.shape[0]),
                                          c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(out))
        _check(rc, "direct_sum_cells")
        return out

    def fft(self, x: np.ndarray, sign: int = -1) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.complex128).ravel()
        out = np.empty_like(x)
        _check(self.lib.or_fft(int(x.shape[0]), _dp(x.view(np.float64)), _dp(out.view(np.float64)), sign), "fft")
        return out

    def fft3(self, a: np.ndarray, sign: int = -1) -> np.ndarray:
        a = np.array(a, dtype=np.complex128, order="C", copy=True)
        if a.ndim != 3 or len(set(a.shape)) != 1:
            raise ValueError("fft3 needs a cubic array")
        _check(self.lib.or_fft3(int(a.shape[0]), _dp(a.view(np.float64)), sign), "fft3")
        return a

    def kernel_pad(self, n: int, dx: float, self_coeff: float = SELF_COEFF) -> np.ndarray:
        p = 2 * n
        k = np.empty((p, p, p), dtype=np.float64)
        _check(self.lib.or_kernel_pad(n, dx, self_coeff, _dp(k)), "kernel_pad")
        return k

    def green_hat(self, n: int, dx: float, self_coeff: float = SELF_COEFF) -> np.ndarray:
        p = 2 * n
        g = np.empty((p, p, p), dtype=np.complex128)
        _check(self.lib.or_green_hat(n, dx, self_coeff, _dp(g.view(np.float64))), "green_hat")
        return g

    def fft_conv_kernel(self, rho: np.ndarray, kpad: np.ndarray, dx: float, G: float = 1.0) -> np.ndarray:
        rho = _cube(rho)
        n = rho.shape[0]
        kpad = np.ascontiguousarray(kpad, dtype=np.float64)
        if kpad.shape != (2 * n,) * 3:
            raise ValueError("kpad must be (2N)^3")
        phi = np.empty_like(rho)
        _check(self.lib.or_fft_conv_kernel(n, dx, G, _dp(kpad), _dp(rho), _dp(phi)), "fft_conv_kernel")
        return phi

    def fft_conv(self, rho: np.ndarray, dx: float, G: float = 1.0, self_coeff: float = SELF_COEFF) -> np.ndarray:
        rho = _cube(rho)
        phi = np.empty_like(rho)
        _check(self.lib.or_fft_conv(rho.shape[0], dx, G, self_coeff, _dp(rho), _dp(phi)), "fft_conv")
        return phi

    # cells of spacings dx, dy, dz along x, y, z
    def cell_average_inv_r(self, dx: float, dy: float, dz: float) -> float:
        return self.lib.or_cell_average_inv_r(float(dx), float(dy), float(dz))

    def kernel_value3(self, di: int, dj: int, dk: int, dx: float, dy: float, dz: float,
                      self_coeff: float = SELF_COEFF) -> float:
        return self.lib.or_kernel_value3(int(di), int(dj), int(dk), float(dx), float(dy), float(dz), float(self_coeff))

    def direct_sum3(self, rho: np.ndarray, dx: float, dy: float, dz: float, G: float = 1.0,
                    self_coeff: float = SELF_COEFF) -> np.ndarray:
        rho = _cube(rho)
        phi = np.empty_like(rho)
        _check(self.lib.or_direct_sum3(rho.shape[0], dx, dy, dz, G, self_coeff, _dp(rho), _dp(phi)), "direct_sum3")
        return phi

    def direct_sum_cells3(self, rho: np.ndarray, cells: Sequence[Sequence[int]], dx: float, dy: float, dz: float,
                          G: float = 1.0, self_coeff: float = SELF_COEFF) -> np.ndarray:
        rho = _cube(rho)
        c = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, 3))
        out = np.empty(c.shape[0], dtype=np.float64)
        rc = self.lib.or_direct_sum_cells3(rho.shape[0], dx, dy, dz, G, self_coeff, _dp(rho), int(c.shape[0]),
                                           c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(out))
        _check(rc, "direct_sum_cells3")
        return out

    def kernel_pad3(self, n: int, dx: float, dy: float, dz: float, self_coeff: float = SELF_COEFF) -> np.ndarray:
        p = 2 * n
        k = np.empty((p, p, p), dtype=np.float64)
        _check(self.lib.or_kernel_pad3(n, dx, dy, dz, self_coeff, _dp(k)), "kernel_pad3")
        return k

    def fft_conv3(self, rho: np.ndarray, dx: float, dy: float, dz: float, G: float = 1.0,
                  self_coeff: float = SELF_COEFF) -> np.ndarray:
        rho = _cube(rho)
        phi = np.empty_like(rho)
        _check(self.lib.or_fft_conv3(rho.shape[0], dx, dy, dz, G, self_coeff, _dp(rho), _dp(phi)), "fft_conv3")
        return phi

    # boxes of nx x ny x nz cells (arrays [z][y][x]) with spacings dx, dy, dz
    @staticmethod
    def _box(rho: np.ndarray) -> np.ndarray:
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        if rho.ndim != 3:
            raise ValueError("rho must be a 3D [z][y][x] array")
        return rho

    def direct_sum_box(self, rho: np.ndarray, dx: float, dy: float, dz: float, G: float = 1.0,
                       self_coeff: float = SELF_COEFF) -> np.ndarray:
        rho = self._box(rho)
        nz, ny, nx = rho.shape
        phi = np.empty_like(rho)
        _check(self.lib.or_direct_sum_box(nx, ny, nz, dx, dy, dz, G, self_coeff, _dp(rho), _dp(phi)),
               "direct_sum_box")
        return phi

    def direct_sum_cells_box(self, rho: np.ndarray, cells: Sequence[Sequence[int]], dx: float, dy: float,
                             dz: float, G: float = 1.0, self_coeff: float = SELF_COEFF) -> np.ndarray:
        rho = self._box(rho)
        nz, ny, nx = rho.shape
        c = np.ascontiguousarray(np.asarray(cells, dtype=np.int32).reshape(-1, 3))
        out = np.empty(c.shape[0], dtype=np.float64)
        rc = self.lib.or_direct_sum_cells_box(nx, ny, nz, dx, dy, dz, G, self_coeff, _dp(rho), int(c.shape[0]),
                                              c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dp(out))
        _check(rc, "direct_sum_cells_box")
        return out

    def fft3_box(self, a: np.ndarray, sign: int = -1) -> np.ndarray:
        a = np.ascontiguousarray(a, dtype=np.complex128).copy()
        if a.ndim != 3:
            raise ValueError("a must be a 3D [z][y][x] array")
        pz, py, px = a.shape
        _check(self.lib.or_fft3_box(px, py, pz, _dp(a.view(np.float64)), int(sign)), "fft3_box")
        return a

    def kernel_pad_box(self, nx: int, ny: int, nz: int, dx: float, dy: float, dz: float,
                       self_coeff: float = SELF_COEFF) -> np.ndarray:
        k = np.empty((2 * nz, 2 * ny, 2 * nx), dtype=np.float64)
        _check(self.lib.or_kernel_pad_box(nx, ny, nz, dx, dy, dz, self_coeff, _dp(k)), "kernel_pad_box")
        return k

    def fft_conv_box(self, rho: np.ndarray, dx: float, dy: float, dz: float, G: float = 1.0,
                     self_coeff: float = SELF_COEFF) -> np.ndarray:
        rho = self._box(rho)
        nz, ny, nx = rho.shape
        phi = np.empty_like(rho)
        _check(self.lib.or_fft_conv_box(nx, ny, nz, dx, dy, dz, G, self_coeff, _dp(rho), _dp(phi)),
               "fft_conv_box")
        return phi

    @staticmethod
    def rel_l2(a, ref):
        return rel_l2(a, ref)

    @staticmethod
    def rel_max(a, ref):
        return rel_max(a, ref)


def variant(so_path: str) -> Oracle:
    """An :class:`Oracle` bound to another build of ``oracle.c`` (used by the
    tests that plant mistakes in the oracle to check that the pins catch them)."""
    return Oracle(_bind(ctypes.CDLL(so_path)))


def build_variant(out_path: str, defines: Sequence[str] = ()) -> str:
    cmd = ["gcc", "-std=c11", "-O2", "-fopenmp", "-fPIC", "-shared", *[f"-D{d}" for d in defines],
           "-o", out_path, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    return out_path


_default = Oracle()
set_threads = _default.set_threads
get_threads = _default.get_threads
kernel_value = _default.kernel_value
direct_sum = _default.direct_sum
direct_sum_cells = _default.direct_sum_cells
fft = _default.fft
fft3 = _default.fft3
kernel_pad = _default.kernel_pad
green_hat = _default.green_hat
fft_conv_kernel = _default.fft_conv_kernel
fft_conv = _default.fft_conv
cell_average_inv_r = _default.cell_average_inv_r
kernel_value3 = _default.kernel_value3
direct_sum3 = _default.direct_sum3
direct_sum_cells3 = _default.direct_sum_cells3
kernel_pad3 = _default.kernel_pad3
fft_conv3 = _default.fft_conv3
direct_sum_box = _default.direct_sum_box
direct_sum_cells_box = _default.direct_sum_cells_box
fft3_box = _default.fft3_box
kernel_pad_box = _default.kernel_pad_box
fft_conv_box = _default.fft_conv_box


def rel_l2(a: np.ndarray, ref: np.ndarray) -> float:
    """||a - ref||_2 / ||ref||_2 over all cells."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm((a - ref).ravel()) / np.linalg.norm(ref.ravel()))


def rel_max(a: np.ndarray, ref: np.ndarray) -> float:
    """max|a - ref| / max|ref|."""
    a = np.asarray(a, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.abs(a - ref).max() / np.abs(ref).max())
