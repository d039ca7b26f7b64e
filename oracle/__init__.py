"""FP64 CPU oracle for one soft-sphere DEM timestep -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the benchmark's CPU
baseline may import this package.  It shares no code with the HIP library.
"""
