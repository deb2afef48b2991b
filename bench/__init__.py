"""Measurement drivers beside bench.py: the K sweep at the paper's shapes,
the 16-bit arg-max agreement table, the RFA shift sweep, the iterative loop
on the 100k-particle workload and the uneven-stack batch benchmark.  Each
prints JSON lines; run them from the repository root as ``python -m
bench.<name>``.  None of them is imported by the library."""
