"""Plain FP64 CPU oracle for the space-time IgA heat-equation solver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark may import this package; the HIP library and
its Python binding never do, and the two share no code.  Every function
cites the passage of the paper it follows; where the paper is silent or
garbled the reading taken is stated in the docstring.
"""
