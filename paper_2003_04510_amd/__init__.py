"""MI355X-native full-RNS CKKS (HEAAN) HE Mul, and the paper's own non-RNS
HE Mul on big-integer coefficients (BigContext).

The computation runs in the HIP library libhe_mi355x.so (C ABI, declared in
include/he_mi355x.h).  This package only marshals arguments: PyTorch supplies
device memory and streams.  There is no CPU fallback: if the library is not
built, importing the binding raises.
"""
from .binding import (Batch, BatchGroup, BigContext, Ciphertext, Context, HeBusy, HeError, Server, load_library,  # noqa: F401
                      workload_primes)
