"""MI355X-native per-vertex graphlet orbit counting (orbits 0-72).

The compute path is the HIP library ``liborbit_hip.so`` built from
``csrc/``; :mod:`paper_1911_10616_amd.orbit` is its thin ctypes binding.
Importing this package does not load the library: use
``from paper_1911_10616_amd import orbit``.
"""
__all__ = ["graphgen", "orbit"]
