"""Plain FP64 CPU oracle for the RaftGP hot path (test infrastructure only).

This package is the slow, obviously-correct reference that the HIP path is
checked against.  It is test infrastructure: only the test-suite, the smoke
check and the CPU-baseline leg of the benchmark may import it.  It never
imports the HIP library and the HIP library never uses it.

Modules (each function cites the passage of the paper it follows):

* ``philox``     -- Philox4x64-10 counter-based generator (Salmon et al. 2011).
* ``fmath``      -- own FP64 ln / sincos(2*pi*u) / Box-Muller, basic IEEE ops only.
* ``graph``      -- CSR validation, degrees, 2e (problem statement, Sec. II).
* ``projection`` -- Gaussian random projection Y = X^q Theta (Sec. III-A, Eq. 5).
* ``gcn``        -- random GCN propagation (Sec. III-B, Eq. 6).
* ``kmeans``     -- nested k-means++ seeding (exponential race) and Lloyd.
* ``scores``     -- modularity (Eq. 3), NCut (Eq. 1), model selection, NMI.
* ``hierarchical`` -- local modularity (Eq. 7) and hierarchical model selection (Alg. 1).
* ``sbm_sample`` -- fast sampling from the degree-corrected SBM (Sec. IV, Alg. 2).
* ``streaming``  -- incremental embedding update for new edges (Sec. III-D).
* ``modloss``    -- relaxed modularity loss tr(S^T B S) and its adjoint.
* ``pipeline``   -- the whole path end to end.

Parity status: every function is pinned by a ``-m "not gpu"`` test against a
closed form, an invariant, a library routine or brute force, except where a
module header says "parity unpinned".
"""
