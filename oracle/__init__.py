"""FP64 CPU oracle for the hierarchical view-factor radiosity path.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports, links or calls
this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code, header,
table or constant generator with the HIP path; the only common inputs are
the seeded generators in ``workloads/``.

Contents (each function cites the passage of the paper it follows):

* ``geometry``     facet centroid / unit normal / area from triangles (Sec. 3.1-3.2)
* ``viewfactor``   dense centroid-rule view factors, eq. (10); row sums and the
                   closed-cavity row scaling, eqs. (32)-(34)
* ``clustering``   Algorithm 1 (index tree) and Algorithm 2 (block tree) with the
                   admissibility condition of Sec. 4.2
* ``aca``          adaptive cross approximation (Sec. 4.3, eq. (30)) with the
                   block-wise stopping rule eq. (31); H-matrix assembly and the
                   block-wise product of Sec. 5.2
* ``radiosity``    reflection matrix eq. (11), emission eq. (4), dense LU solve,
                   facet flux eq. (12)
* ``closed_forms`` two infinite gray plates (Sec. 2.2), projected-sphere and
                   aligned-parallel-squares closed forms
* ``transient``    lumped backward-Euler radiative exchange (analogue of Sec. 3.3)
* ``matfree``      the dense definition at large n: products with the
                   centroid-rule entries evaluated on the fly (plain C,
                   ``vf_matfree.c``) and GMRES in place of LU
* ``hlu``          hierarchical block LU of the reflection matrix (Sec. 5.1)
                   and its forward / backward substitution (Sec. 5.2)
* ``fe``           finite-element coupling (Sec. 3.1-3.4): P1 surface
                   elements, P, R_bar, S = P^T R_bar P, implicit Euler with
                   Newton on the nodal residual

Where the paper is silent the readings are fixed in the module docstrings.
"""
