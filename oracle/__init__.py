"""FliX batch-semantics oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import anything in this package.  The product path (the
``paper_2604_16725_amd`` package and its HIP library) never does.
"""
