"""MI355X-native PLAST-P bank-versus-bank hot path.

Subpackages are imported lazily: ``synth`` (seeded synthetic banks) has no GPU
dependency, ``binding`` loads the HIP library (``libplast_hip.so``) and fails
loudly when it is missing.
"""

__all__ = ["synth", "binding", "params"]
