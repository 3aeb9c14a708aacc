"""MI355X-native solid lattice-Boltzmann primal + discrete-adjoint library.

The compute path lives in the HIP library built from csrc/ (loaded lazily by
`paper_2609_31347_amd.slbm`); `paper_2609_31347_amd.inputs` holds the seeded
synthetic problem data.
"""
__all__ = ["inputs", "slbm"]
