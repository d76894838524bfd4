"""CPU FP64 oracle for the IPN / AMIPN hot path.

TEST INFRASTRUCTURE ONLY: tests/, the smoke check and the bench's CPU-baseline
leg may import it; the product library (paper_2510_04170_amd) never does, and
this package never imports the product.  See oracle.rfm for the method and
oracle.philox for the sketch's random numbers.
"""
