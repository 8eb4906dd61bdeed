"""FP64 CPU oracle for the closed-shell (T) energy correction.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path;
the only thing both sides use is the seeded input generator in ``synth``.

Contents
--------
closed_shell
    The closed-shell (T) energy as a plain loop over unique occupied
    triples i <= j <= k (section 2.4.2 of the paper, Eqs. 2-7, with the
    readings of its garbled equations listed in that module's docstring).
virtual_loop
    The same energy as a plain loop over unique virtual triples a <= b <= c
    with tensors over the occupied indices (the loop order of the paper's
    (T) iteration); pinned to the spin-orbital definition and to
    ``closed_shell``.
spin_orbital
    A brute-force spin-orbital (T) energy from the textbook definition
    (Raghavachari et al. 1989; Crawford & Schaefer, Rev. Comp. Chem. 14,
    2000), used only on tiny systems to pin the closed-shell oracle.
mp2
    The closed-shell MP2 energy (the paper's MP2 equation) with
    density-fitted integrals, and the spin-orbital MP2 definition that pins
    it.

Every function works in IEEE FP64.  Parity status: every function is
pinned (see tests/test_oracle_pins.py,
tests/test_oracle_virtual_pins.py and tests/test_oracle_mp2_pins.py); no function here is "parity
unpinned".
"""
from .closed_shell import (  # noqa: F401
    t_energy,
    triple_energy,
    triple_table,
    w_tensor,
    v_tensor,
)
from .spin_orbital import spinorb_t_energy  # noqa: F401
from .virtual_loop import t_energy_virtual_loop, virtual_triple_energy, virtual_triple_table  # noqa: F401
from .mp2 import mp2_energy, pair_energies, spinorb_mp2_energy  # noqa: F401
