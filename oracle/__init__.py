"""CPU oracle for the FMM-accelerated Burton-Miller collocation BEM.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call, link or run anything in this package;
only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
use it.  It shares no code with the HIP library: the only common module is
``workloads`` (seeded mesh and random-input generators, which hold none of the
boundary-element arithmetic).

It computes, plainly and slowly, in complex128:

* ``bem``    - element geometry, the Helmholtz kernel and its normal
               derivatives, the quadrature rules, near-singular and self
               integrals, and the exact discrete Burton-Miller operator and
               its adjoint (dense or by row/column blocks);
* ``mie``    - the rigid-sphere plane-wave series (closed-form reference);
* ``tree``   - Morton keys, the sorted order and the uniform-depth octree
               with its neighbour (U) and interaction (V) lists, in Python
               integers (the bit-exact reference);
* ``solve``  - restarted GMRES (modified Gram-Schmidt), dense LU solves, the
               field representation at exterior points, the objective
               J = sum |p(x_obs)|^2 and its discrete-adjoint gradient;
* ``fem``    - linear-tetrahedron stiffness and mass of the elastic body, the
               boundary coupling and the Schur form of the BEM-FEM system
               (Eqs. fem_2, renritupu, kousokuu, GMRES);
* ``elastic_sphere`` - plane-wave scattering by an elastic sphere in a
               fluid, the partial-wave series from the governing equations
               (the analytic check of Sec. 3.1).

Paper anchors (Isakari, Kondo, Takahashi, Matsumoto, "A level-set-based
topology optimisation for acoustic-elastic coupled problems with a fast
BEM-FEM solver"): the boundary integral equation of Sec. 2.3 (Eq. danseibie2)
with G = exp(ik|x|)/(4 pi |x|), piecewise-constant triangles with collocation
(Sec. 2.3), the block system (Eq. renritupu) whose acoustic block is I/2 - D,
the iterative solution of Eq. (GMRES), and the objective of Eq. (obj).
Readings where the paper is silent (quadrature rule, collocation point,
hypersingular finite part, Burton-Miller coupling, admittance condition,
Morton order, tree rule) are stated in the docstring of the function that
uses them.

Parity status: every function here is pinned by a test in
``tests/test_oracle_*.py`` against a closed form, an independent numerical
method, an invariant or a library routine.
"""
