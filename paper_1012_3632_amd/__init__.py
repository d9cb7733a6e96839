"""MI355X (gfx950) fluctuating lattice Boltzmann library.

The fused per-site D2Q9/D3Q19 step (pull streaming, moment transform,
relaxation with fluctuation-dissipation noise, optional square-gradient force)
runs in hand-written HIP kernels behind the C ABI of include/flb.h
(libflb.so, built in-tree by ``python paper_1012_3632_amd/build.py``).
torch is used for device memory and streams only.
"""

from .sim import (Batch, Params, Simulation, field_spectrum, lattice_tables,  # noqa: F401
                  noise_normals, noise_words, query_sizes)
