"""MI355X-native Super-Droplet Method (SDM) collision-coalescence.

The hot path (per-cell Philox keys, LDS-staged segmented sort, pairing,
scaled probabilities, integer collision counts and the multiplicity /
attribute update, plus per-cell moments) runs in hand-written HIP kernels for
gfx950 behind the C ABI declared in ``include/sdm.h`` (``libsdm.so``).

  ``binding``  ctypes marshalling of that ABI (same names as the C calls)
  ``inputs``   seeded synthetic initial states (no step arithmetic)
  ``serving``  continuous batching of box simulations over the ABI

Importing this package loads nothing; ``binding`` loads ``libsdm.so`` and
raises if it is missing.
"""
__all__ = ["binding", "inputs", "serving"]
