"""MI355X-native RACIPE ensemble integrator (GRiNS, arXiv 2503.18356).

Submodules:
  inputs   -- seeded synthetic topologies (no method arithmetic)
  racipe   -- Python binding of the C-ABI library (librac.so)
The binding is imported lazily so that topology generation works without the
native library.
"""
__all__ = ["inputs", "racipe"]
