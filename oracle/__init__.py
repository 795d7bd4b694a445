"""Oracle: plain, slow, FP64 CPU implementation of the space-time HDG + AIR
method (Sivas, Southworth, Rhebergen, arXiv 2010.11130).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import or call anything here.
The HIP library never uses it and shares no code with it; the only code the
two sides share is the ``workloads`` package of seeded problem inputs.

Modules
  quad      collapsed Gauss-Jacobi simplex rules (scipy's Gauss-Jacobi nodes)
  basis     equispaced Lagrange bases on simplices (product formula)
  hdg       mesh topology, element blocks of the bilinear form (Section 2.3),
            static condensation (Section 2.5), assembly, Dirichlet
            elimination, facet-block scaling, reconstruction, L2 error
  air       lAIR algebraic multigrid setup and V-cycles (Section 3, Section 4
            solver settings) and the transposed cycle
  krylov    flexible GMRES with right preconditioning
  adjoint   adjoint solve and gradients of a facet misfit w.r.t. f and nu
  drivers   whole solves: all-at-once and slab-by-slab (Sections 2.2, 2.4)

Every function states the passage of the paper it follows.  Functions that
no independent pin covers say "parity unpinned" in their docstring.
"""
