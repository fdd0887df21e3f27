"""Plain FP64 CPU oracle for environment-recycled imaginary-time TEBD.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or
executes this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may use it.  It shares no code with the
HIP library; the two meet only through the seeded generators in ``tninputs``.

The oracle is written from Phien, McCulloch and Vidal, "Faster convergence
of imaginary time evolution tensor network algorithms by recycling the
environment" (arXiv:1411.0391), in NumPy/SciPy float64, using library
routines (``svd``, ``eigh``, ``solve``, ``expm``, ``eig``) for every
factorization and no blocking, fusion or reordering beyond what the paper
states.  Where the paper is silent, the module docstrings name the reading
taken.

Modules
-------
gates      Trotter gates, iMPO and iPEPO (Sec. V A, Eq. (iMPO1); Sec. VI A).
imps       1D: transfer-matrix fixed points, truncation (Eq. (EqCanoPQ1)),
           canonical form (Sec. III A), gauge fixing (Sec. III B),
           renormalized gate and recycling (Sec. V B), energy.
ctmrg      2D corner transfer matrix environment (Sec. VI B, Fig. 21).
peps       iPEPS reduced density matrices and energy, canonical form
           (Sec. IV A, Eqs. (17)-(20)) and gauge fixing (Sec. IV B, Eq. (25)).
fu         full-update bond environment and the variational (ALS) truncation
           (Sec. VI B, Eqs. (var), (var1)); recycling driver (Sec. VI C).
grad       energy of a single-site iPEPS after a fixed number of CTMRG
           iterations, and its central finite-difference gradient.
"""
