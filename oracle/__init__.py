"""FP64 CPU oracle for DADE inside an IVF scan.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import or call anything in this package.
The product path (the HIP library and its Python binding) never does, and the
two share no code: this package imports nothing from the product package.

Plain, slow, obviously-correct NumPy in float64.  Each function cites the part
of the paper it follows:

* ``pca``        -- the data-aware orthogonal transform (Lemma 1, Lemma 2,
                    Eqs. (10)-(12)): centring, E[XX^T], eigenvectors sorted by
                    descending eigenvalue, the transformed objects.
* ``estimator``  -- the scaled estimate of Eq. (13), the deviation bound eps_d
                    of Eq. (14) estimated from sampled data pairs, and the
                    hypothesis test of the "Dimension Expansion with Hypothesis
                    Testing" subsection.
* ``dco``        -- Algorithm 1 (one DADE distance comparison) and FDScanning.
* ``ivf``        -- k-means lists, probe order and the IVF scan with a size-K
                    max-heap (end of the Methodology section), under a round
                    schedule that fixes which threshold each DCO sees.
* ``knn``        -- brute-force K nearest neighbours (ground truth).
* ``lowp``       -- rounding of stored coordinates to BF16 / FP16 and the
                    rerank margin for the low-precision index (not in the
                    paper; the reading is documented where it is defined).

Parity status per function is listed in each module header.  Every function
here is pinned by a ``-m "not gpu"`` test against something other than itself.
"""
