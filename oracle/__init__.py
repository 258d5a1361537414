"""FP64 CPU oracle of the ray-traced Gaussian renderer.

TEST INFRASTRUCTURE ONLY. Only tests/, the smoke check and the CPU-baseline
leg of the benchmark may import it; the product path never does.
"""
