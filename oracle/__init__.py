"""FP64 CPU oracle for the finite-difference micromagnetic hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package; only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP path:
it is a plain, slow, obviously correct restatement of the paper's equations
(MicroMagnetic.jl paper, sections "Micromagnetics", "LLG equation",
"Miscellaneous") in NumPy/SciPy double precision.

Modules
-------
newell   cell-averaged demagnetisation tensor (Newell closed form near,
         Gauss-Legendre quadrature of its defining double volume integral far)
fields   exchange, interfacial DMI, uniaxial anisotropy, Zeeman and demag
         fields, energies and the Landau-Lifshitz right-hand side
potential  demag field through the magnetic scalar potential (vertex potential, edge differences)
cells    cell-based Ms, A and D (harmonic means) and empty cells
dp45     adaptive Dormand-Prince 5(4) with unit-sphere projection
neb      nudged-elastic-band force and relaxation iteration

Parity status: every function here is pinned by tests under tests/ against
closed forms, invariants, brute force or library routines, except the NEB
force, whose physical barrier values are "parity unpinned" (the paper prints
no NEB formulas; see the neb module header).
"""
MU0 = 4e-7 * 3.141592653589793238462643383279502884  # vacuum permeability, exact by convention
GAMMA_DEFAULT = 2.21e5  # m/(A s), the gyromagnetic ratio printed with the macrospin test
