"""Plain, slow FP64 CPU oracle for the brick-local random-walker solve.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The HIP product
path (``paper_2103_09564_amd``) never imports it, and this package imports
nothing from the product path: the two share no code.  The only module both
sides use is ``synth`` (seeded synthetic inputs, none of the method's
arithmetic).

Everything here follows Drees, Eilers & Jiang, "Hierarchical Random Walker
Segmentation for Large Volumetric Biomedical Images" (arXiv 2103.09564):

* ``rw``         -- Section III-B: Gaussian edge weights, graph Laplacian,
                    the Dirichlet problem L_UU x_U = -L_UM x_M, and its
                    solution (sparse direct, dense Cholesky, Jacobi-PCG as in
                    Section V); multi-class one-vs-rest (Section III-B).
* ``brute``      -- brute-force pins of the solve: absorbing Markov chain and
                    Monte-Carlo random walkers (the random-walker
                    interpretation of Section III-B).
* ``hierarchy``  -- Section III-A (LOD pyramid), Section IV-A/B (eqs. 1-3:
                    border seeds from the parent, neighbourhood expansion),
                    Section IV-D (pruning hom/dt/cfl, warm start, ancestor
                    fallback), Section IV-E (incremental labelling).
* ``adjoint``    -- gradient of a loss on x with respect to beta and the
                    intensities, by the adjoint of the Dirichlet problem
                    (derived from Section III-B; the paper itself has no
                    gradient).

All arithmetic is float64.  Inputs may be float32 (they are cast).
"""

from . import rw, brute, hierarchy, adjoint  # noqa: F401
