"""MI355X-native DMRG compression step for quantum-circuit simulation.

Hot path: the compression step of Ayral et al. (two-site variant, one layer
per step) as a HIP library for gfx950 behind a C ABI (``include/mps_dmrg.h``).

* ``paper_2207_05612_amd.circuits`` -- seeded synthetic circuit generators;
* ``paper_2207_05612_amd.mps``      -- the Python binding of the C ABI;
* ``paper_2207_05612_amd.build``    -- hipcc build of ``libmpsdmrg.so``.

Importing the package has no side effects; ``mps.load_library()`` loads the
HIP library and raises if it is not built.
"""
