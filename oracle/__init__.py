"""CPU oracle for the SecPE encrypted Argmax (arXiv 2502.00847).

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports this; only
``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline leg of
``bench.py`` may load it.  It shares no code with the GPU library.

Three tiers:
  * ``sim.t0_*``   the plain definition: argmax of the prompt-summed logits.
  * ``sim.t1_*``   Algorithm 1 in FP64 on real slot vectors with the polynomial
                   Sign, separating approximation error from encryption noise.
  * ``ckks.Oracle``  a plain C RNS-CKKS (128-bit products reduced with '%',
                   textbook NTT) that the GPU ciphertexts must match bit for bit.
"""
from .build import build_oracle, oracle_lib_path  # noqa: F401
