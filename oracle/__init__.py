"""Reference oracle for the temporal-adaptive finite-volume Euler path.

TEST INFRASTRUCTURE ONLY: a plain, slow FP64 CPU implementation that the GPU
library is checked against.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the GPU
library and never imports it.

``oracle.core`` wraps the C oracle (``oracle.c``), ``oracle.mlp_ref`` is the
FP64 reference of the small p* network.
"""
