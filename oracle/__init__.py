"""CPU oracle for the half-range lattice Boltzmann Couette solver.

TEST INFRASTRUCTURE: imported only by tests/, __graft_entry__.smoke() and the CPU-baseline leg of
bench.py.  The GPU product path never imports, loads or calls anything here.
"""
