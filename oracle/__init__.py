"""CPU oracle for exact data-series k-NN search (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import anything from this package.  The search
library (``paper_2212_13297_amd``) never imports, links or calls it, and it
never imports the library: the two share no code.  Inputs come from the seeded
generators in ``paper_2212_13297_amd.datagen``, which hold none of the
method's arithmetic.

Contents (every function cites the passage of Hercules, PVLDB 15(10) 2022,
that it follows):

* ``brute``     -- FP64 brute-force k-NN (C/OpenMP ``knn_brute.c`` and a numpy
                   twin for tiny inputs): the plain k-NN definition.
* ``summaries`` -- FP64 PAA, Gaussian breakpoints, iSAX words, LB_SAX, EAPCA
                   segment statistics, node synopses, LB_EAPCA, and the
                   mean/std midpoint H-split.
* ``search``    -- a serial FP64 run of the paper's exact search (approximate
                   seed over L_max leaves, candidate leaves by LB_EAPCA,
                   candidate series by LB_SAX, refinement with early
                   abandoning) over a leaf partition built by ``summaries``.

Precision is FP64 throughout; inputs are the canonical float32 series.
Parity status of each function is recorded in its docstring; every function
here is pinned by ``tests/test_oracle_*.py`` against closed forms, invariants,
library routines for special cases, brute force on tiny inputs, or the worked
split example the paper prints.
"""
