"""Plain CPU reference ("oracle") for the time-harmonic Maxwell hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call or execute anything in this package; only the
test suite, the smoke check and the CPU-baseline leg of the benchmark do.

Everything here is written from the paper's mathematics (Beuchler, Kinnewig,
Wick, "Parallel domain decomposition solvers for the time harmonic Maxwell
equations", arXiv 2105.11993) in complex128 with NumPy/SciPy:

* ``fe``       reference Nedelec basis, quadrature, element matrices (Sec. 2, eq. (3))
* ``mesh``     box meshes, entity/DoF numbering, boundary sets, partitions (eq. (5))
* ``system``   global assembly, Dirichlet data, lifting, direct solves (eqs. (1)-(4))
* ``gmres``    plain right-preconditioned GMRES (Sec. 3.2, eq. (11))
* ``ddm``      impedance-transmission domain decomposition (eqs. (6)-(10))
* ``adjoint``  objective J = int_T |E|^2 and its exact discrete gradient in mu
* ``closed_form`` the normally incident plane wave and its exact 1D discrete solution

The oracle shares no code with the GPU path.  Conventions (basis, orientation,
DoF order, quadrature, Dirichlet projection) are stated in each module's
docstring and implemented independently on both sides.
"""
