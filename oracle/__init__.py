"""FP64 CPU oracle of the DMRG compression step -- TEST INFRASTRUCTURE ONLY.

Plain, slow, obviously correct NumPy complex128 code that follows the paper
(Ayral et al., "A density-matrix renormalization group algorithm for simulating
quantum circuits with a finite fidelity") step by step.  It shares no code with
the GPU library; the only thing both sides import is the seeded input
generator ``paper_2207_05612_amd.circuits``.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from this package.  The product path never
does.
"""
from . import dmrg, statevector, philox, chaotic  # noqa: F401
