"""CPU oracle for the UniHENN hot path.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark import this package.  It shares no code with the product
library (paper_2402_03060_amd) and never imports it; the only module both sides
use is `workloads` (seeded input generators, no arithmetic of the method).
"""
