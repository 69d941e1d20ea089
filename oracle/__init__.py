"""FP64 CPU oracle for the space-time hp-DG residual of the time-dependent
Maxwell equations (Lilienthal, Schnepp, Weiland, arXiv 1307.5310).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The library
(``paper_1307_5310_amd``) never imports, links or calls this package, and this
package imports nothing from the library; the two share only the seeded input
generators in ``synth``, which hold no discretisation arithmetic.

What it computes is the plain definition: the slab bilinear form B_h = C_h + S_h
of the weak formulation (Section 2.5, eq. bilinearform:C; Section 4.1,
eq. bilinearform:S and weakform_stabilized) evaluated on every trial/test pair
of the tensor-product bases of Section 5.1, by full Gauss quadrature, assembled
into dense local blocks and applied block by block (Section 5.2 only reorganises
these integrals).  Pieces:

* ``basis``   1D orthonormal / integrated Legendre functions and the time and
              derivative tables, all by quadrature (Section 5.1, eq. def:ilegendre),
              and the tables of bisected slab intervals (local time steps,
              Section 2.2) with the projection of S_h.
* ``geometry``trilinear element maps and the face topology of a hex mesh.
* ``dg``      dense local element and face matrices, slab blocks, the residual
              (Section 5, eq. residual), the load, the energy (eq.
              stability:energydef), sparse slab assembly and solves.
* ``brute``   a separately written physical-space assembler for tiny meshes:
              covariantly mapped basis functions, chain-rule curls, physical
              normals, Newton inversion for neighbour traces, S_h from its
              definition.  It pins ``dg``.
* ``fields``  analytic fields (TE101, manufactured solutions, cavity modes,
              Gaussian pulse) and their projections.

Parity status: every function here is pinned by a ``-m "not gpu"`` test except
the non-affine mass matrix beyond the shared Gauss rule (n_q = p + 2 points per
direction), whose agreement with the exact integral is a quadrature error,
reported, not claimed: parity unpinned for that part.
"""
