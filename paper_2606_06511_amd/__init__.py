"""MI355X-native triangle-triangle intersection energy (TTIE) hot path.

The compute path is the HIP library ``libttie.so`` built from ``csrc/`` for gfx950 and
reached through the thin ctypes binding in :mod:`paper_2606_06511_amd.ttie`.  Importing the
package itself loads nothing; the binding loads the library on first use and raises if it
is missing (there is no CPU fallback).
"""

__all__ = ["workloads", "ttie"]
