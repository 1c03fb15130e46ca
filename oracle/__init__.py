"""PairHMM forward-algorithm oracle: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It is independent of the product
library: it computes its own priors from the Phred bytes and evaluates the
forward recurrences of the paper's Section 2 (eq. 1-4) in FP64 on the host.

Contents
--------
``phmm_oracle.c`` (loaded through ctypes)
    row-order forward pass (optionally with per-row power-of-two
    rescaling), the anti-diagonal order, and the row-level formulation of
    Section 3.1 (eq. 7) evaluated literally.
``exact.py``
    pure-Python path enumeration and exact rational evaluation, used only to
    pin the C oracle on tiny inputs.
``genotype.py``
    diploid genotype likelihoods from a read x haplotype likelihood matrix
    (the genotyping step after the PairHMM), plain FP64 definition.
"""
from .oracle import (  # noqa: F401
    NREC, build_oracle, priors, forward_probs, forward_one, forward_pairs,
    forward_antidiag_probs, forward_rowform_probs, lib_path,
)
from .genotype import genotype_region, genotype_batch, best_genotype  # noqa: F401
