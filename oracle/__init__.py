"""CPU oracle for discord search -- TEST INFRASTRUCTURE, not part of the product.

Only the tests, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library
(``paper_1901_00155_amd``): the two meet only in the seeded inputs of
``paper_1901_00155_amd.workloads``, which hold none of the method's arithmetic.

Contents (each function cites the passage of the paper it follows):
  ``discord``          brute-force FP64 discord (C, definition of section 2.1)
  ``rows_nn``          exact nearest non-self match of chosen rows (C)
  ``pair_d2``          eq. (1) squared for one pair (C)
  ``stats``            eq. (2) mean / standard deviation (C, two-pass)
  ``witness_check``    FP64 certificate that a claimed discord is the argmax (C)
  ``sax_words``        eqs. (3), (4), (9): PAA -> SAX -> word id per row (C)
  ``np_discord``       independent NumPy brute force (all pairs at once)
  ``int_discord``      exact-integer enumerator in pure Python ints
  ``alg1``             abandoning search (Algorithm 1) with any visiting order
  ``phidd``            the same search in PhiDD's visiting orders (Algorithms 2-4)
  ``breakpoints``, ``freq_cand``, ``index_word``   SAX helpers of section 3.1
"""
from .oracle import *  # noqa: F401,F403
