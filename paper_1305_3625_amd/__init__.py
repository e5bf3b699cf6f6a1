"""MI355X-native FFT-convolution conjugate-gradient solver.

The solver (HIP kernels for gfx950 behind the C ABI in ``include/fftcg.h``)
is in ``libfftcg.so``; ``binding`` is its Python face.  Importing this package
loads nothing; ``binding.load()`` loads the library and raises if it is not
built.
"""

__version__ = "0.1.0"
