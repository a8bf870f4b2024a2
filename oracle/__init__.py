"""FP64 CPU oracle for the DDC products of column-generation VMAT optimisation.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference written from the paper (Tian et al., "Multi-GPU implementation of a
VMAT treatment plan optimization algorithm", arXiv:1503.01721).  Only the test
suite, the smoke check and the benchmark's CPU-baseline leg may import it; the
product path (the HIP library and its Python binding) never does, and this
package never imports the product path.  It shares no code with it: inputs
come as plain NumPy arrays from the seeded synthetic-workload generator.

Modules
-------
products   dose z = D x, price p = D^T g, aperture DDC vectors (Eqs. 3, 5)
objective  one-sided quadratic objective F, its gradient, curvature (Eq. 1, 4)
aperture   aperture selection by exhaustive interval enumeration (Sec. 2.2.2)
bb         Barzilai-Borwein master-problem solver with the subspace bound
           handling of Eqs. (7)-(10), in D-form and in DA-form (Eq. 6)
colgen     the column-generation loop (Sec. 2.1)
machine    gantry-speed bounds from leaf motion and speed change, and the
           rate box of every aperture (Eq. 2, Eq. 6)

All floating point is float64.
"""
