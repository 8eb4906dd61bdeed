"""MI355X (gfx950) closed-shell (T) energy: HIP kernels behind a C ABI.

The computation lives in libbqc.so (built from csrc/ by ``build.py``); this
package holds only the ctypes binding of include/bqc.h.
"""
from .binding import (  # noqa: F401
    BqcError,
    Server,
    PRECISIONS,
    batch_footprint,
    footprint,
    header_functions,
    last_error,
    lib,
    mp2_energy_df,
    noalloc_batch,
    num_triples,
    runtime_versions,
    t_energy,
    t_energy_batch,
    t_energy_df,
    t_energy_noalloc,
    t_energy_plain,
)

__all__ = ["BqcError", "Server", "PRECISIONS", "batch_footprint", "footprint", "header_functions", "last_error", "lib",
           "mp2_energy_df", "noalloc_batch", "num_triples", "runtime_versions", "t_energy", "t_energy_batch", "t_energy_df",
           "t_energy_noalloc", "t_energy_plain"]
