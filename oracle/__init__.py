"""FP64 CPU oracle of the haemoglobin-estimation path.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's CPU
baseline use it; the GPU library never does.
"""
