"""MI355X (gfx950) DG2 flood-model time step.

``paper_2010_02003_amd.dg2``      ctypes binding of the C ABI (include/dg2.h)
``paper_2010_02003_amd.workloads`` seeded synthetic inputs
``paper_2010_02003_amd.build``     builds libdg2.so with hipcc

Importing the package does not touch the GPU; creating a ``Sim`` loads the
library and fails loudly if it is missing.
"""
from .dg2 import DG2Error, Sim, load_library, sim_from_scenario  # noqa: F401
