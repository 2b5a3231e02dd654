"""CPU oracle of the cluster-preserving correction (test infrastructure only).

``oracle.correct`` and friends wrap the plain C reference in
``pcc_oracle.c`` through ctypes.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg use this package; the GPU library never does.
"""
from .oracle import (  # noqa: F401
    MODE_VP, MODE_SC, MODE_HF, NONE, SAFE, PB, PC,
    build, lib_path, constants, pairs, classify, components, select,
    correct, decode, fof_labels, OracleResult,
)
