"""CPU oracle for the column-wise RNS-CKKS inference path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check and the CPU
baseline leg of ``bench.py`` may import this package.  The product path (the
HIP library and its Python binding) never imports, links or calls it, and it
imports nothing from the product: the two share no code, tables or constant
generators.  Inputs that both sides consume come from ``synthetic_inputs``,
which holds no arithmetic of the method.

Layout:
  ckks_oracle.c   textbook modular arithmetic, NTT, base conversion, ChaCha20
                  and samplers, built with gcc into liboracle.so
  _clib.py        ctypes loader (builds the .so with gcc when it is missing)
  ckks.py         RNS-CKKS scheme in the coefficient domain
  layers.py       the column-wise schedules and their FP64 plaintext layers

Parity status per function is listed in the header of each module.
"""
from .ckks import (Params, Context, Ciphertext, ExtCiphertext, Plaintext, Keys, SwitchingKey,  # noqa: F401
                   gen_primes, find_psi, cdt_table, security_bound, PRESETS)
