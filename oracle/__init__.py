"""CPU oracle of the RB-TAI Active Flux step -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU-baseline leg
may import this package.  The product library never calls it.
"""
