"""FP64 CPU oracle for the two-centre multipole method (test infrastructure only).

Only tests/, the smoke check and the benchmark's CPU-baseline leg import this package.
It shares no code with the HIP implementation in paper_0704_1672_amd/.
"""
from .oracle import (  # noqa: F401
    load, moments, energy, coulomb, centroid, radius, pose, ylm, threej, trunc_bound,
    complex_to_packed, packed_to_complex, pair_energy_from_atoms,
    energy_grad, energy_coeffs, atom_forces, pair_forces, energy_sensitivity, SQUARE, TRIANGULAR,
)
