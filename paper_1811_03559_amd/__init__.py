"""MI355X (gfx950) recursive SPIKE banded solver.

The solver itself is the HIP library ``libspike.so`` (C ABI in
``include/spike.h``); ``paper_1811_03559_amd.spike`` is its ctypes binding and
``paper_1811_03559_amd.inputs`` the seeded synthetic input generators.
"""
