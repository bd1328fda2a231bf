"""CPU oracle for the device data-sharing runtime -- TEST INFRASTRUCTURE.

``ref``: plain definitions of the loop results (C, fp64, exact sums).
``sim``: a contention-group simulator of the master/worker protocol and the
team stack (frames, placement, LIFO pops, reductions, invariants).
``footprint``: the paper's static shared-memory and occupancy arithmetic.

Only the tests, the package smoke check and the benchmark's CPU-baseline leg
may use this package; the GPU path never imports it.
"""
