"""FP64 CPU oracle for the neural receiver and its classical judge.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the product path (the HIP library and
its Python binding) never does.  It shares no code with the GPU path: inputs are
passed in as arrays, and its random draws use its own Philox implementation.
"""
from . import philox, nr, slot_sim, receiver, cgnn  # noqa: F401
