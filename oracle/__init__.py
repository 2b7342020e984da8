"""FP64 CPU oracle for the Minimod acoustic_iso_cd hot path.

TEST INFRASTRUCTURE ONLY: the correctness reference that the GPU library is
checked against.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark import this package; the product path never does.

`oracle.c_oracle` wraps the plain-C implementation (minimod_oracle.c, built
with the Makefile beside it); `oracle.tiny` is a second, independent numpy
implementation used to cross-check the C one on tiny grids.
"""
from . import c_oracle, tiny  # noqa: F401
