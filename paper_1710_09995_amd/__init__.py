"""MI355X-native multi-block structured-grid residual / RK3 library.

The compute path lives in ``libcfd.so`` (hand-written HIP for gfx950 behind a
C ABI, declared in ``include/cfd.h``); ``binding`` marshals arguments to it.
``cases`` builds seeded synthetic inputs.  Importing this package loads
nothing; ``binding.lib()`` loads the shared library on first use and raises
if it is missing.
"""
__version__ = "0.1.0"
