"""Plain double-precision CPU oracle of the hydro step (test infrastructure).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. It shares no code with the GPU library.
"""
