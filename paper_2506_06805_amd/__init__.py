"""MI355X-native CD/FNS IP-EOM-CCSD hot path.

The compute path lives in the HIP library `libfnscc.so` (built from `csrc/`)
and is reached through the thin ctypes binding in `fnscc.py`.  Importing the
package does not load the library; `paper_2506_06805_amd.fnscc` does, and it
raises if the library is missing.
"""
__all__ = ["synth"]
