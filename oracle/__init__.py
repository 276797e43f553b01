"""Plain CPU oracle of the ternary flip-graph random walk.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU
baseline leg of the benchmark may import it; the product library never does.
"""
