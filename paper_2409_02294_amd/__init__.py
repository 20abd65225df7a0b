"""Free-space Poisson solver by FFT convolution for one MI355X (gfx950).

The solve runs in hand-written HIP kernels behind the C ABI of
``include/ps.h`` (``libps.so``); :mod:`.solver` is its Python binding and
:mod:`.inputs` the seeded synthetic-density generator.  Importing the package
loads nothing; the library is loaded on first use of :mod:`.solver`.
"""
__all__ = ["solver", "inputs", "build"]
