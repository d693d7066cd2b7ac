"""CPU FP64 oracle for the mixed Gaussian/triangle rasterizer and the
proxy-mesh deformation transfer.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
GPU path is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never
does.  It shares no code with the GPU library: every formula here is written
out from the paper (single-pass rasterization, Section 3.2, Eq. 1-11;
deformation transfer, Section 3.3.2, Eq. 12-13) and from the 3DGS
conventions that the paper builds on.
"""
