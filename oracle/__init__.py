"""CPU oracle for the streamed GWAS GLS path (test infrastructure only).

Imported only by tests/, __graft_entry__.smoke() and bench.py's cpu_baseline
leg.  Shares no code with the HIP library.
"""
