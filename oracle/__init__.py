"""FP64 CPU oracle of the filtering / Favre / SGS-tensor path and of the learned closure.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline leg of the
benchmark are the only callers. The product library never imports, links or runs
anything here, and nothing here imports the product library. The oracle is plain
numpy in float64, written from the paper's definitions (see each docstring).
"""
from . import fields, mlp  # noqa: F401
