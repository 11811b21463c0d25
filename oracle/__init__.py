"""FP64 CPU oracle of the lattice kinetic Kohn-Sham relaxation.

Test infrastructure only: the test suite, the smoke check and the benchmark's
CPU-baseline leg may import it; the GPU library never does.
"""
