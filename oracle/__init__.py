"""CPU oracle of the solid-LBM primal, adjoint and gradient.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg.  Never by the HIP package.
"""
