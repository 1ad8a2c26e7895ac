"""Plain FP64 CPU oracle of the periodic SWG volume-integral-equation method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports or calls this
package: only the tests, the smoke check in __graft_entry__.py and the bench's CPU-baseline leg
do.  It shares no code with the HIP library (no kernels, tables, helpers or
constant generators); the only common inputs are the seeded meshes and
permittivities from the input-generator module.

It follows the paper's method in its own order and notation:
  * VIE in the polarisation (Sec. 2.1, Eq. 1), SWG basis with Galerkin testing
    (Sec. 2.1, Eq. 2), contrast kappa = (eps_r - 1)/eps_r;
  * two-dimensional periodic Green's function with the Bloch phase of the
    incident plane wave (Sec. 2.2, Eqs. 3-4), evaluated by the Ewald split
    into spatial and spectral series (Sec. 2.2);
  * block partition by material domain and the block-diagonal preconditioner
    (Sec. 2.3, Eqs. 5-6), GMRES (Sec. 3);
  * absorbed power Im(eps)|E|^2 per domain (Sec. 3, Eq. 7).

Modules:
  quadrature  point rules on tetrahedra and triangles
  pgf         Ewald periodic Green's function, plus direct/spectral lattice sums
  potentials  closed-form 1/R and R integrals over triangles and tetrahedra
  topology    SWG faces, periodic pairing, orientation, unknown order, near pairs
  vie         impedance matrix, right-hand side, solves, absorptance, R/T
  fresnel     transfer-matrix reflection/transmission of a homogeneous slab

Pins for every function live in tests/ (marked "not gpu").
"""
