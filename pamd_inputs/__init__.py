"""Seeded synthetic inputs shared by the oracle tests and the GPU library tests.

Holds no force-field, integrator or resampling arithmetic."""
from .systems import (System, bead_chain, gaussian_chain, spring_pair, make_peptide,
                      c1_system, c2_system, c4_systems, C4_SIZES, geometric_schedule,
                      KB_KJ, KE_KJ, DIELECTRIC_VACUUM, DIELECTRIC_4R, N_TYPES)
