"""FP64 CPU oracle for the FLARE B2 force field evaluation (energies, forces, uncertainties).

TEST INFRASTRUCTURE ONLY. Nothing on the product path imports, links or executes
anything in this package: only the tests, the smoke check and the CPU-baseline leg
of the benchmark use it. It shares no code with the HIP path; the two meet only in
the seeded input generators, which hold none of the method's arithmetic.

Every function is the plain definition from the paper, written for clarity over speed:
  * local environment rho_i = all neighbours within the cutoff (Section V.B);
  * ACE B2 descriptors from radial functions x real spherical harmonics, normalised
    d_i = d~_i / |d~_i| (Section V.B, Fig. 3);
  * mapped mean and variance as quadratic forms d^T beta d and d^T gamma d (Eq. 1, Eq. 2);
  * forces as -dE/dr formed through the explicit descriptor gradient (the direct
    route that the force reordering of Section V.B avoids), and by central differences;
  * velocity-Verlet NVE and Nose-Hoover NVT for the short MD checks, hydrogen
    coordination numbers and reaction events of the production runs (Section VI.A).

Readings of what the paper leaves open (radial basis, cutoff shape, packing order,
one model per central species, ...) are listed in the design notes and in the
docstrings of `hyper.py`.
"""
