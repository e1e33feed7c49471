"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This package holds only input synthesis: the LDA generative process used to
plant topics (paper, Appendix "Simulation Data Generation Process"), splitting
a corpus into CSR batches, and the seeded initial CP factors.  It contains none
of the method's arithmetic (no moments, whitening, gradients or recovery), so
both the FP64 oracle and the HIP path can be fed from it without sharing code.
"""
from .lda_corpus import (Corpus, CorpusSpec, SPECS, generate, iter_batches,
                         init_phi, make_csr_rows, slice_specs)

__all__ = ["Corpus", "CorpusSpec", "SPECS", "generate", "iter_batches",
           "init_phi", "make_csr_rows", "slice_specs"]
