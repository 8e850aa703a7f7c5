"""FP64 CPU oracle for exemplar-based clustering.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the CPU
baseline of the benchmark. The HIP product path never imports it.

``ebc_oracle`` holds the literal NumPy definitions (small sizes);
``ref`` wraps the plain-C loops of ``ebc_ref.c`` (same definitions, fast
enough for the benchmark sizes).
"""
from . import ebc_oracle  # noqa: F401
from . import ref  # noqa: F401
