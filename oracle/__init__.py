"""CPU oracle for adaptive-multilevel BDDC (plain FP64 NumPy/SciPy).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it to check the GPU library; the product path never imports it
and it shares no code with the GPU library.
"""
