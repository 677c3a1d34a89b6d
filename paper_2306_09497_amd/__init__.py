"""MI355X-native Parareal/MGRIT integration of the rotating shallow-water
equations on the sphere (spherical-harmonic IMEX propagator, arXiv 2306.09497).

The compute path lives in the HIP shared library ``libpint.so`` (sources in
``csrc/``, C ABI in ``include/pint.h``); ``pint`` is its ctypes binding.
"""
