"""MI355X-native multi-level foreground estimation (arXiv 2006.14970).

The compute path is the HIP library ``libfge.so`` built from ``csrc/`` for gfx950; the Python
binding in :mod:`paper_2006_14970_amd.fge` only marshals torch tensors to its C ABI.  Importing
this package does not load the library; the binding loads it on first use and raises if it is
missing.
"""
__all__ = ["fge", "synth"]
