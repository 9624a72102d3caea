"""FP64 CPU oracle for Schwarz-factorised stochastic determinant-ratio estimation.

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow, obviously correct
reference against which the HIP library is checked.  Only the test-suite, the
smoke check and the benchmark's CPU-baseline leg may import, call, link or run
anything under ``oracle/``.  The product path never routes through it and
shares no code with it (no kernels, headers, helpers, tables or constants).

Contents
  lattice.py    geometry: site indexing, neighbours, time boundary sign,
                Schwarz blocks, black/white colouring, the projector P
  dirac.py      chiral gamma matrices, the clover field and the assembled
                sparse Wilson-clover operator D(m) in the mass normalisation
  schwarz.py    D_bb, D_ww, D_bw, D_wb, the Schur complement and its
                P-restricted form and inverse (Sec. 1, Eq. 1)
  nested.py     nested domain decomposition (Sec. 2.2): the Schur complement of the
                Dirichlet operator of one colour's outer blocks with respect to inner
                blocks, and the total log W with exact inner block determinants
  estimator.py  the two-flavour noise estimator of Eq. (3), W_gl of Eq. (8) and the
                one-flavour estimator of Eq. (11)
                with mass interpolation, log-domain combination, variances
  derivative.py derivatives of the exponents and of log W_gl with respect to kappa2
                and the links, by extrapolated central differences (exact solves)
  cref.py       ctypes wrapper of c/ddref.c, a matrix-free FP64 C version of
                the operator, block solves and estimator for lattices too large
                for the assembled matrix
Readings of points the paper leaves open are listed in each module header.
"""
