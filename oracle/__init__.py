"""FP64 CPU oracle for the lattice Boltzmann scheme with relative velocities.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package; only the tests, the smoke check
and the CPU-baseline leg of the benchmark do.  It shares no code, tables or
constants with the HIP library: velocity sets, weights, polynomial bases and
every formula are written out here a second time, from the paper.

Contents
--------
lattices   velocity sets, weights and moment bases (paper section 1.3, and a
           reading for three dimensions, where the paper has none)
scheme     Oracle A: one time step as defined in section 1.2 (shifted moment
           matrix M(u~) evaluated from the polynomials, LU solve per node)
mrt        Oracle C: the d'Humieres MRT step of section 1.1, written separately
geier      Oracle D: the cascaded g-vector form of Appendix B
adjoint    Oracle E: discrete adjoint / tangent of Oracle A's step (FP64)
fast       Oracle B: the same definition in plain C with OpenMP (liboracle_fast)
stability  Oracle F: linear (von Neumann) stability about a uniform flow, from
           the Jacobian of Oracle E's step and the transport phases

lattices.with_basis builds a lattice with a run-time polynomial basis given as
term lists (used to check the library's run-time bases).
"""
