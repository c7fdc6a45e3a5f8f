"""CPU oracle (test infrastructure only).

Plain, slow, obviously correct CPU implementations of what the GPU library
computes, each citing the passage of the paper it follows. Only the test
suite, the smoke check and the CPU-baseline leg of the benchmark import this
package; the GPU library never does, and the two share no code.
"""
